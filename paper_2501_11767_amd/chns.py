"""Thin ctypes binding of libchns.so (the C-ABI in include/chns.h).

Only argument marshalling lives here: every step of the solve runs in the
library's HIP kernels.  Device buffers are torch CUDA tensors (PyTorch-ROCm
provides device memory and streams); calls run on torch's current stream.
The binding raises if the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libchns.so")

OK, WNOCONV, EINVAL, ENOMEM, EHIP, ESTATE, EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5
MODEL_CH, MODEL_CH_AC, MODEL_TERNARY, MODEL_QUATERNARY = 0, 1, 2, 3
BLOCK_CH, BLOCK_AC, BLOCK_NS = 0, 1, 2
OP_M, OP_K, OP_C, OP_CH, OP_AC, OP_X, OP_L, OP_NS, OP_VX, OP_AP = range(10)
KERNEL_CHEB32, KERNEL_CHEB64, KERNEL_CH_BLOCK, KERNEL_DCGS_DOTS, KERNEL_DCGS_UPDATE, KERNEL_MG_FINE = range(6)
KERNEL_NAMES = {
    KERNEL_CHEB32: "k_stencil7<float, float, 2>",
    KERNEL_CHEB64: "k_stencil7<double, double, 2>",
    KERNEL_CH_BLOCK: "CH operator (k_ch_block; k_ch_dots with the dot pass)",
    KERNEL_DCGS_DOTS: "k_dcgs_dots",
    KERNEL_DCGS_UPDATE: "k_dcgs_update",
    KERNEL_MG_FINE: "k_vtile_pipe (finest-level tile passes; k_vtile in FP64)",
}
F64, MIXED = 0, 1
MODELS = {"ch": MODEL_CH, "ch_ac": MODEL_CH_AC, "ternary": MODEL_TERNARY, "quaternary": MODEL_QUATERNARY}

EXPORTS = [
    "chns_default_opts", "chns_create", "chns_destroy", "chns_set_params", "chns_assemble", "chns_set_density",
    "chns_matrix_shape", "chns_get_matrix", "chns_spmv", "chns_precond_apply",
    "chns_krylov_solve", "chns_step_rhs", "chns_diagnostics", "chns_diagnostics_noalloc",
    "chns_timestep", "chns_last_error",
    "chns_assemble_transposed", "chns_timestep_adjoint", "chns_ledger_start", "chns_ledger_read",
    "chns_batch_create", "chns_batch_destroy", "chns_batch_offsets", "chns_batch_timestep",
    "chns_batch_tune", "chns_batch_tuned", "chns_batch_set_worklist", "chns_batch_set_graph_budget",
    "chns_batch_precond_apply",
    "chns_batch_last_error",
]


class Mesh(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("model", ct.c_int32), ("boundary", ct.c_int32), ("dim", ct.c_int32),
                ("length", ct.c_double)]


BOUNDARY_PERIODIC, BOUNDARY_NOFLUX = 0, 1
BOUNDARIES = {"periodic": BOUNDARY_PERIODIC, "noflux": BOUNDARY_NOFLUX}


POT_QUARTIC, POT_FLORY_HUGGINS = 0, 1
# the paper's Flory-Huggins values for the full model (sizes, chi, saturated fractions)
FLORY_HUGGINS = dict(potential=POT_FLORY_HUGGINS, fh_nsize=(5.0, 5.0, 1.0), fh_chi=(4.0, 0.3, 0.3),
                     fh_phisat=(1e-8, 1e-8, 1e-6))


class Params(ct.Structure):
    _fields_ = [(k, ct.c_double) for k in
                ("eps", "tau", "mobility", "evap_rate", "viscosity", "alpha", "rho")] + \
               [("potential", ct.c_int32), ("truncate", ct.c_int32), ("fh_nsize", ct.c_double * 3),
                ("fh_chi", ct.c_double * 3), ("fh_phisat", ct.c_double * 3),
                ("var_density", ct.c_int32), ("ns_picard", ct.c_int32), ("rho_pure", ct.c_double * 3),
                ("ns_picard_tol", ct.c_double), ("top_flux", ct.c_double), ("flux_inf", ct.c_double),
                ("beta_phase", ct.c_double * 4)]

    def __init__(self, *args, **kw):
        arrays = {k: kw.pop(k) for k in ("fh_nsize", "fh_chi", "fh_phisat", "rho_pure", "beta_phase") if k in kw}
        super().__init__(*args, **kw)
        for k, v in arrays.items():
            setattr(self, k, (ct.c_double * len(v))(*v))


class SolveOpts(ct.Structure):
    _fields_ = [("rtol", ct.c_double), ("atol", ct.c_double), ("restart", ct.c_int32),
                ("maxiter", ct.c_int32), ("precision", ct.c_int32), ("mg_cycles", ct.c_int32),
                ("mg_pre", ct.c_int32), ("mg_post", ct.c_int32), ("mg_coarse", ct.c_int32),
                ("mg_lmax", ct.c_double), ("mg_rho_cut", ct.c_double)]


class SolveInfo(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("restarts", ct.c_int32), ("converged", ct.c_int32),
                ("status", ct.c_int32), ("bnorm", ct.c_double), ("res0", ct.c_double),
                ("res_true", ct.c_double), ("ms", ct.c_double), ("passes", ct.c_int32),
                ("change", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)


class TorchAllocator:
    """Device memory of the library's contexts from PyTorch's caching
    allocator (chns_create / chns_batch_create allocator callbacks).  The
    counters record every call the library makes, so that a caller can check
    that no entry point allocates after creation."""

    alloc_calls = 0
    free_calls = 0

    @staticmethod
    def _alloc(nbytes, _ctx):
        import torch
        TorchAllocator.alloc_calls += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    @staticmethod
    def _free(ptr, _ctx):
        import torch
        TorchAllocator.free_calls += 1
        torch.cuda.caching_allocator_delete(int(ptr))


# module-level references keep the ctypes thunks alive as long as the library
_ALLOC_THUNK = ALLOC_FN(TorchAllocator._alloc)
_FREE_THUNK = FREE_FN(TorchAllocator._free)


def _allocator(use_torch):
    if use_torch:
        return _ALLOC_THUNK, _FREE_THUNK
    return ALLOC_FN(), FREE_FN()  # NULL: the library's own hipMalloc / hipFree


class Fields(ct.Structure):
    _fields_ = [("phi", ct.c_void_p * 3), ("mu", ct.c_void_p * 4), ("Phi_v", ct.c_void_p),
                ("vel", ct.c_void_p), ("p", ct.c_void_p)]


_lib = None


def lib():
    """Load libchns.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: run __graft_entry__.build() (or "
                           "python -m paper_2501_11767_amd.build) first")
    # torch first: it carries its own HIP runtime (same SONAME), which the
    # library then binds to, so device pointers and streams are shared.
    import torch  # noqa: F401
    L = ct.CDLL(LIBPATH)
    vp, i32, dbl = ct.c_void_p, ct.c_int32, ct.c_double
    L.chns_default_opts.argtypes = [ct.POINTER(SolveOpts)]
    L.chns_default_opts.restype = None
    L.chns_create.argtypes = [ct.POINTER(Mesh), ct.POINTER(Params), ALLOC_FN, FREE_FN, vp,
                              ct.POINTER(vp)]
    L.chns_destroy.argtypes = [vp]
    L.chns_set_params.argtypes = [vp, ct.POINTER(Params)]
    L.chns_assemble.argtypes = [vp, vp, vp, vp]
    L.chns_set_density.argtypes = [vp, vp, vp, vp]
    L.chns_matrix_shape.argtypes = [vp, i32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64),
                                    ct.POINTER(ct.c_int64)]
    L.chns_get_matrix.argtypes = [vp, i32, vp, vp, vp, vp]
    L.chns_spmv.argtypes = [vp, i32, i32, i32, dbl, vp, dbl, vp, vp]
    L.chns_precond_apply.argtypes = [vp, i32, i32, ct.POINTER(SolveOpts), vp, vp, vp]
    L.chns_krylov_solve.argtypes = [vp, i32, i32, vp, vp, ct.POINTER(SolveOpts),
                                    ct.POINTER(SolveInfo), vp]
    L.chns_step_rhs.argtypes = [vp, ct.POINTER(Fields), vp, vp, vp, vp]
    L.chns_diagnostics.argtypes = [vp, ct.POINTER(Fields), ct.POINTER(ct.c_double), vp]
    L.chns_diagnostics_noalloc.argtypes = [vp, ct.POINTER(Fields), ct.POINTER(ct.c_double), vp]
    L.chns_timestep.argtypes = [vp, ct.POINTER(Fields), ct.POINTER(Fields), i32,
                                ct.POINTER(SolveOpts), ct.POINTER(SolveInfo), vp]
    L.chns_assemble_transposed.argtypes = [vp, vp, vp, vp]
    L.chns_timestep_adjoint.argtypes = [vp, ct.POINTER(Fields), ct.POINTER(Fields), ct.POINTER(Fields),
                                        ct.POINTER(Fields), vp, ct.POINTER(SolveOpts), vp, vp]
    L.chns_ledger_start.argtypes = [vp, i32]
    L.chns_ledger_read.argtypes = [vp, vp, vp, vp]
    L.chns_last_error.argtypes = [vp]
    L.chns_last_error.restype = ct.c_char_p
    L.chns_batch_create.argtypes = [i32, vp, vp, ALLOC_FN, FREE_FN, vp, ct.POINTER(vp)]
    L.chns_batch_destroy.argtypes = [vp]
    L.chns_batch_offsets.argtypes = [vp, vp]
    L.chns_batch_timestep.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, i32, ct.POINTER(SolveOpts),
                                      i32, vp, vp, ct.POINTER(ct.c_double), vp]
    L.chns_batch_tune.argtypes = [vp, ct.c_char_p, vp]
    L.chns_batch_tuned.argtypes = [vp, vp, vp]
    L.chns_batch_set_worklist.argtypes = [vp, i32]
    L.chns_batch_set_graph_budget.argtypes = [vp, i32, i32]
    L.chns_batch_precond_apply.argtypes = [vp, i32, vp, vp, ct.POINTER(SolveOpts), vp]
    L.chns_batch_last_error.argtypes = [vp]
    L.chns_batch_last_error.restype = ct.c_char_p
    for name in EXPORTS:
        if name not in ("chns_default_opts", "chns_last_error", "chns_batch_last_error"):
            getattr(L, name).restype = ct.c_int
    _lib = L
    return L


class ChnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"chns error {code}: {msg}")
        self.code = code


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().chns_default_opts(ct.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t, numel, dtype=None, name="tensor", optional=False):
    """Device pointer of a tensor after checking everything the library
    assumes about it: a contiguous CUDA tensor of `dtype` (float64 unless
    given) with exactly `numel` elements.  The kernels read and write numel
    elements through the pointer, so a short or mistyped tensor would be
    accessed past its end."""
    import torch
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name}: a tensor is required")
    dtype = torch.float64 if dtype is None else dtype
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return ct.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """Owns a chns_ctx for one mesh/model/parameter set.  boundary "periodic"
    (n^2 nodes) or "noflux" (the closed square, (n+1)^2 nodes); length: the
    square's side; dim 3: the cube (n^3 nodes periodic, (n+1)^3 closed; binary
    models)."""

    def __init__(self, n: int, model: str = "ch_ac", torch_alloc: bool = True,
                 boundary: str = "periodic", length: float = 1.0, dim: int = 2, **params):
        self.L = lib()
        self.n, self.model, self.dim = n, model, dim
        self.boundary, self.length = boundary, length
        m = n + 1 if boundary == "noflux" else n  # vertices per side
        self.N = m ** dim
        p = dict(eps=0.02, tau=1e-3, mobility=1.0, evap_rate=0.0, viscosity=1.0, alpha=1e-8,
                 rho=1.0)
        p.update(params)
        self.params = p
        m = Mesh(n=n, model=MODELS[model], boundary=BOUNDARIES[boundary], dim=dim, length=length)
        h = ct.c_void_p()
        af, ff = _allocator(torch_alloc)
        rc = self.L.chns_create(ct.byref(m), ct.byref(Params(**p)), af, ff, None, ct.byref(h))
        if rc != OK:
            raise ChnsError(rc, self.L.chns_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.chns_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise ChnsError(rc, self.L.chns_last_error(self.h).decode())
        return rc

    def set_params(self, **params):
        self.params.update(params)
        self._check(self.L.chns_set_params(self.h, ct.byref(Params(**self.params))))

    def _mu_array(self, mu):
        if mu is None:
            return None
        mu = list(mu)
        k = 4 if self.model == "quaternary" else 3
        if len(mu) != k:
            raise ValueError(f"mu: expected {k} chemical potentials (polymer, NFA, solvent"
                             + (", air)" if k == 4 else ")"))
        self._mu_keep = mu
        return (ct.c_void_p * k)(*[_ptr(t, self.N, name=f"mu[{i}]", optional=True)
                                   for i, t in enumerate(mu)])

    def set_density(self, phi_p, phi_n):
        """rho^k from the phase fields for the next assemble (var_density)."""
        self._check(self.L.chns_set_density(self.h, _ptr(phi_p, self.N, name="phi_p"),
                                            _ptr(phi_n, self.N, name="phi_n"), _stream()))

    def assemble(self, vel=None, mu=None):
        self._check(self.L.chns_assemble(self.h, _ptr(vel, 8 * self.N, name="vel", optional=True),
                                         self._mu_array(mu), _stream()))

    def assemble_transposed(self, vel, mu=None):
        """Transposed operators at the state (vel, mu) (ternary model)."""
        self._check(self.L.chns_assemble_transposed(
            self.h, _ptr(vel, 8 * self.N, name="vel", optional=True), self._mu_array(mu), _stream()))

    def op_size(self, op):
        """Rows (= columns) of an operator of chns_spmv."""
        return {OP_CH: 2 * self.N, OP_NS: 9 * self.N, OP_VX: 4 * self.N}.get(op, self.N)

    def block_size(self, block):
        return {BLOCK_CH: 2 * self.N, BLOCK_AC: self.N, BLOCK_NS: 9 * self.N}[block]

    def matrix(self, op):
        """Download an operator as (rowptr, col, val) numpy arrays."""
        import numpy as np
        r, c, z = ct.c_int64(), ct.c_int64(), ct.c_int64()
        self._check(self.L.chns_matrix_shape(self.h, op, ct.byref(r), ct.byref(c), ct.byref(z)))
        rp = np.zeros(r.value + 1, dtype=np.int32)
        col = np.zeros(z.value, dtype=np.int32)
        val = np.zeros(z.value, dtype=np.float64)
        self._check(self.L.chns_get_matrix(self.h, op, rp.ctypes.data_as(ct.c_void_p),
                                           col.ctypes.data_as(ct.c_void_p),
                                           val.ctypes.data_as(ct.c_void_p), _stream()))
        return rp, col, val, (r.value, c.value)

    def spmv(self, op, x, y, alpha=1.0, beta=0.0, precision=F64, transpose=False):
        import torch
        k, dt = self.op_size(op), (torch.float32 if precision == MIXED else torch.float64)
        self._check(self.L.chns_spmv(self.h, op, precision, int(bool(transpose)), alpha,
                                     _ptr(x, k, dt, "x"), beta, _ptr(y, k, dt, "y"), _stream()))

    def precond(self, block, r, z, opts=None, transpose=False):
        o = opts or default_opts()
        k = self.block_size(block)
        self._check(self.L.chns_precond_apply(self.h, block, int(bool(transpose)), ct.byref(o),
                                              _ptr(r, k, name="r"), _ptr(z, k, name="z"), _stream()))

    def solve(self, block, b, x, opts=None, transpose=False):
        o = opts or default_opts()
        info = SolveInfo()
        k = self.block_size(block)
        self._check(self.L.chns_krylov_solve(self.h, block, int(bool(transpose)), _ptr(b, k, name="b"),
                                             _ptr(x, k, name="x"), ct.byref(o), ct.byref(info),
                                             _stream()))
        return info.as_dict()

    def fields(self, phi=(), mu=(), Phi_v=None, vel=None, p=None) -> Fields:
        """Field set of device pointers (each tensor checked for dtype, device,
        layout and size); the tensors stay referenced by the returned
        structure so they outlive the calls that use it."""
        phi, mu = tuple(phi), tuple(mu)
        if len(phi) > 3 or len(mu) > 4:
            raise ValueError("at most three phase fields and four chemical potentials")
        f = Fields()
        f._keep = (phi, mu, Phi_v, vel, p)
        for i, t in enumerate(phi):
            f.phi[i] = _ptr(t, self.N, name=f"phi[{i}]")
        for i, t in enumerate(mu):
            f.mu[i] = _ptr(t, self.N, name=f"mu[{i}]", optional=True)
        f.Phi_v = _ptr(Phi_v, self.N, name="Phi_v", optional=True)
        f.vel = _ptr(vel, 8 * self.N, name="vel", optional=True)
        f.p = _ptr(p, self.N, name="p", optional=True)
        return f

    def step_rhs(self, fin: Fields, rhs_ch, rhs_ac=None, rhs_ns=None):
        nch = {"ternary": 2, "quaternary": 3}.get(self.model, 1)
        self._check(self.L.chns_step_rhs(self.h, ct.byref(fin), _ptr(rhs_ch, 2 * nch * self.N, name="rhs_ch"),
                                         _ptr(rhs_ac, self.N, name="rhs_ac", optional=True),
                                         _ptr(rhs_ns, 9 * self.N, name="rhs_ns", optional=True), _stream()))

    def diagnostics(self, f: Fields):
        """[mass phi (or phi_p), mass phi_N, mass phi_s, mass Phi_v, energy] (FP64, synchronising)."""
        out = (ct.c_double * 5)()
        self._check(self.L.chns_diagnostics(self.h, ct.byref(f), out, _stream()))
        return [out[i] for i in range(5)]

    def diagnostics_noalloc(self, f: Fields):
        """As diagnostics(), through the entry point that allocates nothing
        (library-owned static device scratch, shared by every call on a GPU)."""
        out = (ct.c_double * 5)()
        self._check(self.L.chns_diagnostics_noalloc(self.h, ct.byref(f), out, _stream()))
        return [out[i] for i in range(5)]

    def ledger_start(self, kernel):
        """Time every launch of kernel class `kernel` (KERNEL_*) from now on; -1 stops."""
        self._check(self.L.chns_ledger_start(self.h, int(kernel)))

    def ledger_read(self):
        """(launches, algorithmic bytes, event ms) since ledger_start."""
        n, b, ms = ct.c_int64(), ct.c_double(), ct.c_double()
        self._check(self.L.chns_ledger_read(self.h, ct.byref(n), ct.byref(b), ct.byref(ms)))
        return n.value, b.value, ms.value

    def timestep_adjoint(self, fin: Fields, fout: Fields, lam_out: Fields, lam_in: Fields, opts=None):
        """lambda^k from lambda^{k+1} (ternary step); returns (rc, dtheta, infos)
        with dtheta = the step's contribution to dL/d(eps, mobility, evap_rate)."""
        import numpy as np
        o = opts or default_opts()
        dth = np.zeros(3)
        infos = (SolveInfo * 4)()
        rc = self._check(self.L.chns_timestep_adjoint(
            self.h, ct.byref(fin), ct.byref(fout), ct.byref(lam_out), ct.byref(lam_in),
            dth.ctypes.data_as(ct.c_void_p), ct.byref(o), infos, _stream()))
        return rc, dth, [i.as_dict() for i in infos]

    def timestep(self, fin: Fields, fout: Fields, nsteps=1, opts=None, nsolves=None):
        o = opts or default_opts()
        per = {"ch": 1, "ch_ac": 2, "ternary": 4, "quaternary": 5}[self.model]
        k = nsolves or per * nsteps
        infos = (SolveInfo * k)()
        rc = self._check(self.L.chns_timestep(self.h, ct.byref(fin), ct.byref(fout), nsteps,
                                              ct.byref(o), infos, _stream()))
        return rc, [i.as_dict() for i in infos]


class Batch:
    """Owns a chns_batch: independent CH + AC instances advanced together."""

    def __init__(self, sizes, params, torch_alloc: bool = True):
        import numpy as np
        self.L = lib()
        self.count = len(sizes)
        self.sizes = [int(n) for n in sizes]
        n = (ct.c_int32 * self.count)(*self.sizes)
        full = []
        for p in params:
            q = dict(eps=0.02, tau=1e-3, mobility=1.0, evap_rate=0.0, viscosity=1.0, alpha=0.0, rho=1.0)
            q.update(p)
            full.append(Params(**q))
        arr = (Params * self.count)(*full)
        h = ct.c_void_p()
        af, ff = _allocator(torch_alloc)
        rc = self.L.chns_batch_create(self.count, ct.cast(n, ct.c_void_p), ct.cast(arr, ct.c_void_p),
                                      af, ff, None, ct.byref(h))
        if rc != OK:
            raise ChnsError(rc, self.L.chns_batch_last_error(None).decode())
        self.h = h
        off = np.zeros(self.count + 1, dtype=np.int64)
        self.L.chns_batch_offsets(self.h, off.ctypes.data_as(ct.c_void_p))
        self.offsets = off
        self.Ntot = int(off[-1])

    def close(self):
        if getattr(self, "h", None):
            self.L.chns_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise ChnsError(rc, self.L.chns_batch_last_error(self.h).decode())
        return rc

    def tune(self, cache_path=None, stream=None):
        s = ct.c_void_p(stream.cuda_stream) if stream is not None else _stream()
        self._check(self.L.chns_batch_tune(self.h, cache_path.encode() if cache_path else None, s))

    def set_worklist(self, grid):
        """Work-list form of the tiled multigrid passes (grid workgroups; 0: one per tile)."""
        self._check(self.L.chns_batch_set_worklist(self.h, int(grid)))

    def tuned(self):
        """(update-pass threads per chunk, dot-pass vectors per launch) in use."""
        a, g = ct.c_int32(), ct.c_int32()
        self._check(self.L.chns_batch_tuned(self.h, ct.byref(a), ct.byref(g)))
        return a.value, g.value

    def set_graph_budget(self, ch_iters, ac_iters):
        """Arnoldi-step budgets of the graph mode (0: maxiter)."""
        self._check(self.L.chns_batch_set_graph_budget(self.h, int(ch_iters), int(ac_iters)))

    def precond(self, block, r, z, opts=None, stream=None):
        """z = P^{-1} r for every instance (block BLOCK_CH or BLOCK_AC, packed fields)."""
        o = opts or default_opts()
        s = ct.c_void_p(stream.cuda_stream) if stream is not None else _stream()
        k = (2 if block == BLOCK_CH else 1) * self.Ntot
        self._check(self.L.chns_batch_precond_apply(self.h, int(block), _ptr(r, k, name="r"),
                                                    _ptr(z, k, name="z"), ct.byref(o), s))

    def calibrate_graph(self, info, margin=0.125, extra=2):
        """Graph budgets from an eager step's iteration counts: the largest
        count of each block plus a relative margin and a few steps."""
        b = [int(x.max()) for x in (info["iters_ch"], info["iters_ac"])]
        self.set_graph_budget(*[k + extra + int(margin * k) for k in b])

    def timestep(self, phi, mu, Phi, nsteps=1, opts=None, use_graph=False, stream=None,
                 out=None, each_from_input=False):
        """Advance in place, or from (phi, mu, Phi) into out = (phi', mu', Phi')."""
        import numpy as np
        o = opts or default_opts()
        dst = out if out is not None else (phi, mu, Phi)
        it = np.zeros(2 * self.count, dtype=np.int32)
        cv = np.zeros(2 * self.count, dtype=np.int32)
        ms = ct.c_double()
        s = ct.c_void_p(stream.cuda_stream) if stream is not None else _stream()
        N = self.Ntot
        rc = self._check(self.L.chns_batch_timestep(
            self.h, _ptr(phi, N, name="phi"), _ptr(mu, N, name="mu"), _ptr(Phi, N, name="Phi"),
            _ptr(dst[0], N, name="out phi"), _ptr(dst[1], N, name="out mu"), _ptr(dst[2], N, name="out Phi"),
            nsteps,
            int(each_from_input), ct.byref(o), int(use_graph),
            it.ctypes.data_as(ct.c_void_p), cv.ctypes.data_as(ct.c_void_p), ct.byref(ms), s))
        return rc, dict(iters_ch=it[:self.count], iters_ac=it[self.count:], conv_ch=cv[:self.count],
                        conv_ac=cv[self.count:], ms=ms.value)
