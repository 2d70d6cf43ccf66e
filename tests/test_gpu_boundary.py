"""The boundary's promises on the GPU: device memory comes from the caller's
allocator (PyTorch's caching allocator through the binding) and only at
creation; the compute entry points allocate nothing; the binding refuses
tensors of the wrong dtype, size or layout before the library sees them; the
library's own hipMalloc mode gives the same results.
"""
import numpy as np
import pytest

from paper_2501_11767_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_11767_amd import chns
    chns.lib()
    return chns


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_context_memory_comes_from_torch_and_only_at_creation(C):
    import torch
    n = 64
    N = n * n
    a0, f0 = C.TorchAllocator.alloc_calls, C.TorchAllocator.free_calls
    before = torch.cuda.memory_allocated()
    ctx = C.Context(n, "ch_ac", eps=0.02, tau=1e-3, mobility=1.0, evap_rate=0.1)
    a1 = C.TorchAllocator.alloc_calls
    assert a1 - a0 > 50  # every matrix, level and Krylov buffer
    assert torch.cuda.memory_allocated() - before > 8 * 40 * 2 * N  # the FGMRES basis at least
    st = inputs.initial_state(n, "ch_ac", 0.5, 7)
    phi, Phi = _dev(st["phi"][0]), _dev(st["Phi_v"])
    mu = torch.zeros_like(phi)
    vel = _dev(inputs.stream_velocity(n, 3, amp=0.02).ravel())
    f = ctx.fields(phi=[phi], mu=[mu], Phi_v=Phi)
    out = [torch.empty_like(phi) for _ in range(3)]
    fo = ctx.fields(phi=[out[0]], mu=[out[1]], Phi_v=out[2])
    # every compute entry point: assembly, products, preconditioners, solves,
    # right-hand sides, steps, diagnostics
    ctx.assemble(vel)
    rch, rac = torch.empty(2 * N, dtype=torch.float64, device="cuda"), torch.empty_like(phi)
    ctx.step_rhs(f, rch, rac)
    x = torch.zeros_like(rch)
    ctx.spmv(C.OP_CH, rch, x)
    ctx.precond(C.BLOCK_CH, rch, x, C.default_opts(precision=C.MIXED))
    info = ctx.solve(C.BLOCK_CH, rch, x.zero_(), C.default_opts(rtol=1e-10))
    assert info["converged"] == 1, info
    info = ctx.solve(C.BLOCK_AC, rac, torch.zeros_like(rac), C.default_opts(rtol=1e-10, precision=C.MIXED))
    assert info["converged"] == 1, info
    ctx.assemble(None)
    rc, _ = ctx.timestep(f, fo, 2, C.default_opts(rtol=1e-10, precision=C.MIXED))
    assert rc == C.OK
    ctx.diagnostics(fo)
    torch.cuda.synchronize()
    assert C.TorchAllocator.alloc_calls == a1, "a compute call allocated device memory"
    assert C.TorchAllocator.free_calls == f0
    ctx.close()
    assert C.TorchAllocator.free_calls - f0 == a1 - a0  # every buffer went back through free_


def test_ternary_context_allocates_only_at_creation(C):
    import torch
    n = 16
    N = n * n
    st = inputs.initial_state(n, "ternary", 0.3, 5)
    ctx = C.Context(n, "ternary", eps=0.05, tau=1e-4, mobility=1.0, evap_rate=0.1, viscosity=1.0,
                    alpha=1e-8, rho=1.0)
    a1 = C.TorchAllocator.alloc_calls
    z = lambda k=N: torch.zeros(k, dtype=torch.float64, device="cuda")
    fin = ctx.fields(phi=[_dev(st["phi"][0]), _dev(st["phi"][1])], mu=[z(), z(), z()],
                     Phi_v=_dev(st["Phi_v"]), vel=_dev(st["vel"].ravel()), p=z())
    fout = ctx.fields(phi=[z(), z()], mu=[z(), z(), z()], Phi_v=z(), vel=z(8 * N), p=z())
    rc, _ = ctx.timestep(fin, fout, 1, C.default_opts(rtol=1e-10))
    assert rc == C.OK
    lam = ctx.fields(phi=[z(), z()], mu=[z(), z(), z()], Phi_v=z(), vel=z(8 * N), p=z())
    ctx.timestep_adjoint(fin, fout, lam, lam, C.default_opts(rtol=1e-10))
    torch.cuda.synchronize()
    assert C.TorchAllocator.alloc_calls == a1
    ctx.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_allocates_only_at_creation(C, use_graph):
    import torch
    sizes = [32, 64, 32]
    prm = [dict(eps=0.03, tau=1e-4, mobility=1.0, evap_rate=0.1),
           dict(eps=0.02, tau=1e-3, mobility=2.0, evap_rate=0.5),
           dict(eps=0.05, tau=1e-5, mobility=0.5, evap_rate=0.05)]
    batch = C.Batch(sizes, prm)
    a1 = C.TorchAllocator.alloc_calls
    N = batch.Ntot
    phi = torch.rand(N, dtype=torch.float64, device="cuda") * 0.02 + 0.39
    Phi = torch.rand(N, dtype=torch.float64, device="cuda")
    mu = torch.zeros_like(phi)
    s = torch.cuda.Stream()
    o = C.default_opts(rtol=1e-9, restart=30, maxiter=200, precision=C.MIXED)
    with torch.cuda.stream(s):
        out = (torch.empty_like(phi), torch.empty_like(mu), torch.empty_like(Phi))
        rc, info = batch.timestep(phi, mu, Phi, 2, o, use_graph=use_graph, stream=s, out=out)
        # new options rewrite the option tables in place
        o2 = C.default_opts(rtol=1e-9, restart=30, maxiter=200, precision=C.F64, mg_pre=1, mg_post=3)
        rc2, _ = batch.timestep(phi, mu, Phi, 1, o2, use_graph=use_graph, stream=s, out=out)
        r = torch.randn(2 * N, dtype=torch.float64, device="cuda")
        batch.precond(C.BLOCK_CH, r, torch.empty_like(r), o, stream=s)
    s.synchronize()
    assert rc == C.OK and rc2 == C.OK, info
    assert C.TorchAllocator.alloc_calls == a1
    batch.close()


def test_binding_rejects_bad_tensors(C):
    import torch
    n = 16
    N = n * n
    ctx = C.Context(n, "ch_ac", eps=0.05, tau=1e-4)
    good = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
    for bad, what in [(torch.zeros(2 * N, dtype=torch.float32, device="cuda"), "dtype"),
                      (torch.zeros(2 * N - 1, dtype=torch.float64, device="cuda"), "elements"),
                      (torch.zeros(4 * N, dtype=torch.float64, device="cuda")[::2], "contiguous"),
                      (torch.zeros(2 * N, dtype=torch.float64), "CUDA")]:
        with pytest.raises(ValueError, match=what):
            ctx.spmv(C.OP_CH, bad, good)
        with pytest.raises(ValueError, match=what):
            ctx.solve(C.BLOCK_CH, good, bad)
    with pytest.raises(ValueError, match="elements"):
        ctx.fields(phi=[torch.zeros(N + 1, dtype=torch.float64, device="cuda")])
    with pytest.raises(ValueError, match="elements"):
        ctx.assemble(torch.zeros(4 * N, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="dtype"):  # mixed products take FP32 vectors
        ctx.spmv(C.OP_M, torch.zeros(N, dtype=torch.float64, device="cuda"),
                 torch.zeros(N, dtype=torch.float32, device="cuda"), precision=C.MIXED)
    ctx.close()


def test_hipmalloc_mode_gives_the_same_solution(C):
    import torch
    n = 32
    N = n * n
    p = dict(eps=0.02, tau=1e-3, mobility=1.0, evap_rate=0.1)
    g = torch.Generator(device="cuda").manual_seed(3)
    b = torch.randn(2 * N, dtype=torch.float64, device="cuda", generator=g)
    xs = []
    for torch_alloc in (True, False):
        a0 = C.TorchAllocator.alloc_calls
        ctx = C.Context(n, "ch_ac", torch_alloc=torch_alloc, **p)
        assert (C.TorchAllocator.alloc_calls > a0) == torch_alloc
        x = torch.zeros_like(b)
        ctx.solve(C.BLOCK_CH, b, x, C.default_opts(rtol=1e-12))
        xs.append(x.cpu().numpy())
        ctx.close()
    assert np.array_equal(xs[0], xs[1])
