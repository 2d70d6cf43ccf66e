"""The C-ABI library loads, exports every entry point the header declares,
and rejects invalid arguments before touching the device (CPU only)."""
import ctypes as ct
import os
import re

import pytest

from paper_2501_11767_amd import chns

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "chns.h")).read()
    return sorted(set(re.findall(r"CHNS_API\s+[\w\s\*]+?\b(chns_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(chns.LIBPATH):
        pytest.skip("library not built")
    return chns.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(chns.EXPORTS)


def test_default_opts(L):
    o = chns.default_opts()
    assert o.rtol == 1e-8 and o.restart == 40 and o.precision == chns.F64
    assert o.mg_pre == 2 and o.mg_post == 2 and o.mg_coarse == 8
    assert o.mg_lmax == 2.1 and o.mg_rho_cut == 0.25


@pytest.mark.parametrize("n,model", [(7, 0), (6, 0), (0, 1), (10000, 1), (16, 9)])
def test_create_rejects_bad_mesh(L, n, model):
    h = ct.c_void_p()
    rc = L.chns_create(ct.byref(chns.Mesh(n, model)), ct.byref(chns.Params(0.02, 1e-3, 1, 0, 1, 0, 1)),
                       chns.ALLOC_FN(), chns.FREE_FN(), None, ct.byref(h))
    assert rc == chns.EINVAL and not h.value
    assert len(L.chns_last_error(None)) > 0


@pytest.mark.parametrize("boundary,length,model,code", [(7, 1.0, 0, -1), (1, -2.0, 0, -1),
                                                         (1, float("nan"), 1, -1), (0, float("inf"), 0, -1)])
def test_create_rejects_bad_domain(L, boundary, length, model, code):
    """Unknown boundary and a side that is not finite and positive."""
    h = ct.c_void_p()
    rc = L.chns_create(ct.byref(chns.Mesh(n=16, model=model, boundary=boundary, length=length)),
                       ct.byref(chns.Params(0.02, 1e-3, 1, 0, 1, 0, 1)), chns.ALLOC_FN(), chns.FREE_FN(), None,
                       ct.byref(h))
    assert rc == code and not h.value
    assert len(L.chns_last_error(None)) > 0


@pytest.mark.parametrize("dim,n,model,boundary", [(4, 16, 0, 0), (-1, 16, 0, 0), (3, 16, 2, 0), (3, 16, 3, 0),
                                                   (3, 16, 2, 1), (3, 130, 1, 0), (3, 6, 0, 0)])
def test_create_rejects_bad_cube(L, dim, n, model, boundary):
    """The cube takes dim 3 with the binary models and 8 <= n <= 128 (checked
    before any device call)."""
    h = ct.c_void_p()
    rc = L.chns_create(ct.byref(chns.Mesh(n=n, model=model, boundary=boundary, dim=dim)),
                       ct.byref(chns.Params(0.02, 1e-3, 1, 0, 1, 0, 1)), chns.ALLOC_FN(), chns.FREE_FN(), None,
                       ct.byref(h))
    assert rc == chns.EINVAL and not h.value
    assert len(L.chns_last_error(None)) > 0


def test_mesh_struct_layout():
    """chns_mesh: n, model, boundary, dim (int32), then length (double) at byte 16."""
    assert ct.sizeof(chns.Mesh) == 24 and chns.Mesh.length.offset == 16 and chns.Mesh.dim.offset == 12


QB = (2e-4, 2e-4, 1e-3, 4e-3)


@pytest.mark.parametrize("model,boundary,kw,code", [
    (3, 0, dict(beta_phase=(1e-3, 1e-3, 0.0, 1.0)), -1),          # a beta not positive
    (3, 0, dict(beta_phase=(1e-3, 1e-3, float("nan"), 1.0)), -1),
    (2, 0, dict(beta_phase=QB), -1),                              # per-phase betas: quaternary only
    (3, 0, dict(beta_phase=QB, potential=1), -1),                 # Flory-Huggins: ternary only
    (3, 0, dict(beta_phase=QB, var_density=1, rho_pure=(1.0, 1.0, 1.0)), -1),
    (1, 0, dict(ns_picard=3), -1)])                               # Picard: flow models only
def test_create_rejects_model_parameters(L, model, boundary, kw, code):
    h = ct.c_void_p()
    p = chns.Params(**dict(dict(eps=0.05, tau=1e-4, mobility=1.0, evap_rate=0.5, viscosity=1.0,
                                alpha=1e-3, rho=1.0), **kw))
    rc = L.chns_create(ct.byref(chns.Mesh(n=16, model=model, boundary=boundary, length=1.0)), ct.byref(p), chns.ALLOC_FN(),
                       chns.FREE_FN(), None, ct.byref(h))
    assert rc == code and not h.value
    assert len(L.chns_last_error(None)) > 0


@pytest.mark.parametrize("boundary,flux,inf", [(0, 1.0, 0.0), (1, float("inf"), 0.0), (1, 1.0, float("nan"))])
def test_create_rejects_bad_top_flux(L, boundary, flux, inf):
    """The top-wall flux exists on the closed square only, with finite values."""
    h = ct.c_void_p()
    p = chns.Params(0.02, 1e-3, 1, 0, 1, 0, 1)
    p.top_flux, p.flux_inf = flux, inf
    rc = L.chns_create(ct.byref(chns.Mesh(n=16, model=1, boundary=boundary, length=10.0)), ct.byref(p), chns.ALLOC_FN(),
                       chns.FREE_FN(), None, ct.byref(h))
    assert rc == chns.EINVAL and not h.value


@pytest.mark.parametrize("bad", [dict(eps=float("nan")), dict(tau=-1.0), dict(mobility=0.0),
                                 dict(rho=float("inf")), dict(viscosity=0.0)])
def test_create_rejects_bad_params(L, bad):
    p = dict(eps=0.02, tau=1e-3, mobility=1.0, evap_rate=0.1, viscosity=1.0, alpha=1e-8, rho=1.0)
    p.update(bad)
    h = ct.c_void_p()
    rc = L.chns_create(ct.byref(chns.Mesh(16, chns.MODEL_CH_AC)), ct.byref(chns.Params(**p)),
                       chns.ALLOC_FN(), chns.FREE_FN(), None, ct.byref(h))
    assert rc == chns.EINVAL and not h.value


def test_null_context_is_rejected(L):
    assert L.chns_destroy(None) == chns.EINVAL
    assert L.chns_spmv(None, 0, 0, 0, 1.0, None, 0.0, None, None) == chns.EINVAL
    assert L.chns_precond_apply(None, 0, 0, None, None, None, None) == chns.EINVAL
    assert L.chns_krylov_solve(None, 0, 0, None, None, None, None, None) == chns.EINVAL


def test_create_rejects_half_an_allocator(L):
    # an allocator without its free function (or the reverse) is refused
    # before any device work
    h = ct.c_void_p()
    p = chns.Params(0.02, 1e-3, 1, 0, 1, 0, 1)
    rc = L.chns_create(ct.byref(chns.Mesh(16, chns.MODEL_CH)), ct.byref(p), chns._ALLOC_THUNK,
                       chns.FREE_FN(), None, ct.byref(h))
    assert rc == chns.EINVAL and not h.value
    n = (ct.c_int32 * 1)(32)
    rc = L.chns_batch_create(1, ct.cast(n, ct.c_void_p), ct.cast(ct.pointer(p), ct.c_void_p),
                             chns.ALLOC_FN(), chns._FREE_THUNK, None, ct.byref(h))
    assert rc == chns.EINVAL and not h.value


def test_binding_checks_tensors_before_any_call():
    # dtype, device, layout and size are checked on the host: a float32 or a
    # short tensor never reaches the library
    import torch
    with pytest.raises(ValueError, match="CUDA"):
        chns._ptr(torch.zeros(4, dtype=torch.float64), 4)
    with pytest.raises(ValueError, match="required"):
        chns._ptr(None, 4)
    assert chns._ptr(None, 4, optional=True) is None
