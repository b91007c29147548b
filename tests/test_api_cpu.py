"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/lbm.h, and rejects invalid arguments before touching the
device. No compute call is made (no GPU here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "lbm.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def _declared3():
    with open(os.path.join(ROOT, "include", "lbm3d.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(lbm3_[a-z_]+)\s*\(", text)))


def test_three_dimensional_header_exported():
    from paper_2009_06404_amd import _lib3d as L3
    lib = L3.lib()
    names = _declared3()
    assert len(names) == len(L3.ENTRY_POINTS) == 17
    for name in names:
        assert hasattr(lib, name), name
    assert set(L3.ENTRY_POINTS) == set(names)


def _init3(**kw):
    from paper_2009_06404_amd import _lib as L
    from paper_2009_06404_amd import _lib3d as L3
    faces = kw.get("faces", (L.LBM_FREE0, L.LBM_RIGID) + (L.LBM_PERIODIC,) * 4)
    thick = kw.get("thick", (0,) * 6)
    prof = kw.get("prof", (None,) * 6)
    bc, keep = L3.make_bc(faces, thick, prof)
    shape = kw.get("shape", (16, 16, 16))
    fake = 0x2000
    return L3.lbm3_init(*shape, kw.get("q", 19), L.LBM_F32, fake, fake, fake, kw.get("tau", 1.0), bc,
                        kw.get("ws", 0x1000), kw.get("ws_bytes", 1 << 34), None)


@pytest.mark.parametrize("kw,msg", [
    (dict(tau=0.5), "tau"),
    (dict(shape=(2, 16, 16)), ">= 3"),
    (dict(faces=(0, 2, 0, 0, 0, 0)), "paired"),
    (dict(faces=(1, 2, 1, 2, 0, 0)), "top and bottom"),
    (dict(faces=(1, 2, 0, 0, 0, 0), thick=(0, 17, 0, 0, 0, 0), prof=(None, [0.1] * 17) + (None,) * 4),
     "sponge"),
    (dict(faces=(1, 2, 0, 0, 0, 0), thick=(0, 2, 0, 0, 0, 0), prof=(None, [0.1, -1.0]) + (None,) * 4),
     "sponge"),
    (dict(ws=0), "workspace"),
    (dict(ws=0x1004), "aligned"),
    (dict(ws_bytes=100), "too small"),
    (dict(q=15), "lattice"),
])
def test_init3_rejects_invalid_arguments(kw, msg):
    from paper_2009_06404_amd import _lib as L
    with pytest.raises(L.LBMError) as ei:
        _init3(**kw)
    assert msg in str(ei.value)


def test_workspace3_size_and_null_context():
    import ctypes as C
    from paper_2009_06404_amd import _lib as L
    from paper_2009_06404_amd import _lib3d as L3
    b32 = L3.lbm3_workspace_bytes(100, 20, 10, 19, L.LBM_F32)
    assert b32 >= 2 * 19 * 128 * 20 * 10 * 4 + 128 * 20 * 10 * 4
    assert L3.lbm3_workspace_bytes(100, 20, 10, 19, L.LBM_F64) > b32
    b27 = L3.lbm3_workspace_bytes(100, 20, 10, 27, L.LBM_F32)
    assert b27 >= 2 * 27 * 128 * 20 * 10 * 4 + 128 * 20 * 10 * 4 and b27 > b32
    for bad in ((2, 5, 5, 19), (5, 5, 2, 19), (5, 5, 5, 15)):
        with pytest.raises(L.LBMError):
            L3.lbm3_workspace_bytes(*bad, L.LBM_F32)
    with pytest.raises(L.LBMError):
        L3.lbm3_workspace_bytes(2048, 2048, 1024, 19, L.LBM_F32)   # > 2^31 cells
    # one z plane of populations must stay below 2 GiB (32-bit byte offsets):
    # 19 x 1024 x 27584 x 4 B fits, one more row of 64-column pitch does not
    assert L3.lbm3_workspace_bytes(27584, 1024, 4, 19, L.LBM_F32) > 0
    with pytest.raises(L.LBMError, match="2 GiB"):
        L3.lbm3_workspace_bytes(27648, 1024, 4, 19, L.LBM_F32)
    with pytest.raises(L.LBMError, match="2 GiB"):
        L3.lbm3_workspace_bytes(16384, 1024, 4, 27, L.LBM_F64)
    lib = L3.lib()
    assert lib.lbm3_step(None, 1) == L.LBM_E_INVALID
    assert lib.lbm3_moments(None, None) == L.LBM_E_INVALID
    assert lib.lbm3_set_tile(None, 6, 0) == L.LBM_E_INVALID
    assert lib.lbm3_set_lean_width(None, 128) == L.LBM_E_INVALID
    assert lib.lbm3_get_lean_width(None, None) == L.LBM_E_INVALID
    assert lib.lbm3_destroy(None) == L.LBM_OK
    t = C.c_int64(0)
    assert lib.lbm3_get_time(None, C.byref(t)) == L.LBM_E_INVALID


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("lbm_init", "lbm_step", "lbm_moments", "lbm_workspace_bytes",
                 "lbm_set_sources", "lbm_set_receivers", "lbm_destroy", "lbm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2009_06404_amd import _lib as L
    lib = L.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(L.ENTRY_POINTS) <= set(_declared())
    assert L.lbm_abi_version() == 1


def test_workspace_size_and_validation():
    from paper_2009_06404_amd import _lib as L
    b32 = L.lbm_workspace_bytes([(128, 128)], L.LBM_F32)
    b64 = L.lbm_workspace_bytes([(128, 128)], L.LBM_F64)
    assert b64 > b32 >= 2 * 9 * 128 * 128 * 4
    # rows are padded to 64 elements
    assert L.lbm_workspace_bytes([(65, 10)], L.LBM_F32) >= 19 * 128 * 10 * 4
    with pytest.raises(L.LBMError):
        L.lbm_workspace_bytes([(2, 10)], L.LBM_F32)
    with pytest.raises(L.LBMError):
        L.lbm_workspace_bytes([(10, 10)], 7)


def test_workspace_refuses_grids_too_wide_for_the_kernels_descriptors():
    """The step kernels address 2-row tiles plus 6 rows of nine population
    runs from one descriptor of 2^31 - 1 bytes: the widest grid has a pitch
    (nx rounded up to 64) of 3728256 columns in FP64, 7456512 in FP32."""
    from paper_2009_06404_amd import _lib as L
    for code, widest in ((L.LBM_F64, 3728256), (L.LBM_F32, 7456512)):
        assert L.lbm_workspace_bytes([(widest, 3)], code) > 0
        with pytest.raises(L.LBMError, match="too wide"):
            L.lbm_workspace_bytes([(widest + 1, 3)], code)


def _init(**kw):
    from paper_2009_06404_amd import _lib as L
    grids = kw.get("grids", [(16, 16)])
    bcs = kw.get("bcs", [(L.LBM_FREE, L.LBM_RIGID, L.LBM_PERIODIC, L.LBM_PERIODIC, -1)])
    sponges = kw.get("sponges", [((0, 0, 0, 0), (None,) * 4)])
    tau = kw.get("tau", 1.0)
    ws = kw.get("ws", 0x1000)
    ws_bytes = kw.get("ws_bytes", 1 << 30)
    fake = 0x2000
    return L.lbm_init(grids, L.LBM_F32, fake, fake, fake, tau, bcs, sponges, ws, ws_bytes, None)


@pytest.mark.parametrize("kw,msg", [
    (dict(tau=0.5), "tau"),
    (dict(tau=float("nan")), "tau"),
    (dict(grids=[(2, 16)]), ">= 3"),
    (dict(bcs=[(0, 1, 0, 0, -1)]), "paired"),
    (dict(bcs=[(0, 0, 1, 1, -1)]), "free surface"),
    (dict(bcs=[(1, 2, 0, 0, 1)]), "rigid_row"),
    (dict(bcs=[(1, 2, 0, 0, 15)]), "rigid_row"),
    (dict(bcs=[(1, 2, 0, 0, 3)], grids=[(16, 4)]), "rigid_row"),
    (dict(sponges=[((0, 17, 0, 0), (None,) * 4)]), "sponge"),
    (dict(ws=0), "workspace"),
    (dict(ws=0x1004), "aligned"),
    (dict(ws_bytes=100), "too small"),
])
def test_init_rejects_invalid_arguments(kw, msg):
    from paper_2009_06404_amd import _lib as L
    with pytest.raises(L.LBMError) as ei:
        _init(**kw)
    assert msg in str(ei.value)
    assert ei.value.code in (L.LBM_E_INVALID, L.LBM_E_NOMEM)


def test_negative_sponge_profile_rejected():
    import numpy as np
    from paper_2009_06404_amd import _lib as L
    prof = np.array([0.1, -0.2, 0.0])
    with pytest.raises(L.LBMError):
        _init(sponges=[((0, 3, 0, 0), (None, prof, None, None))])


def test_null_context_calls_fail_cleanly():
    from paper_2009_06404_amd import _lib as L
    lib = L.lib()
    assert lib.lbm_step(None, 1) == L.LBM_E_INVALID
    assert lib.lbm_moments(None, 0, None) == L.LBM_E_INVALID
    assert lib.lbm_destroy(None) == L.LBM_OK
    assert "null" in L.last_error() or L.last_error() == ""
    sz = C.c_size_t(0)
    t = C.c_int64(0)
    assert lib.lbm_adjoint_workspace_bytes(None, 10, 100, C.byref(sz)) == L.LBM_E_INVALID
    assert lib.lbm_adjoint_begin(None, 10, 100, None, 0) == L.LBM_E_INVALID
    assert lib.lbm_adjoint_set_io(None, 0, None, None, None) == L.LBM_E_INVALID
    assert lib.lbm_adjoint_step(None, 1) == L.LBM_E_INVALID
    assert lib.lbm_adjoint_time(None, C.byref(t)) == L.LBM_E_INVALID
    assert lib.lbm_adjoint_get_state(None, 0, None) == L.LBM_E_INVALID
    assert lib.lbm_adjoint_set_state(None, 0, None) == L.LBM_E_INVALID
    assert lib.lbm_misfit(None, 0, None, None, 0, None) == L.LBM_E_INVALID
    assert lib.lbm_lame_gradient(None, 0, None, None, None, None, None) == L.LBM_E_INVALID
    assert lib.lbm_step_timed(None, 1, None) == L.LBM_E_INVALID
    g = C.c_double(0)
    assert lib.lbm_stability(None, C.byref(g)) == L.LBM_E_INVALID


@pytest.mark.parametrize("nu,tau", [(0.25, 1.0), (0.0, 1.0), (0.33, 1.0), (0.36, 1.0), (0.37, 1.0),
                                    (0.0, 0.55), (0.1, 0.55), (0.3, 0.55), (0.33, 0.6), (0.4, 2.0)])
def test_library_stability_factor_matches_oracle_theory(nu, tau):
    """lbm_vn_growth (the library's own plane-wave step, host code) against
    the largest eigenvalue modulus of the oracle's independently built von
    Neumann matrix on the same wavenumber grid; the oracle's matrix is pinned
    by plane-wave stepping and the Sec. 4 stability claims."""
    from paper_2009_06404_amd import _lib as L
    from oracle import theory as T
    for nk in (17, 33):
        g = L.lbm_vn_growth(nu, tau, nk)
        ref = T.max_growth(nu, tau, n=nk)
        assert abs(g - ref) < 1e-7, (nk, g, ref)
    # the window the library reports against (Sec. 4: nu = 1/4 unconditionally
    # stable; nu = 0.37 unstable at tau = 1; nu = 0.4 unstable for every tau)
    stable = L.lbm_vn_growth(nu, tau, 33) <= 1.0 + 1e-6
    if nu == 0.25:
        assert stable
    if (nu, tau) in ((0.37, 1.0), (0.4, 2.0), (0.0, 0.55)):
        assert not stable


def test_stability_factor_rejects_bad_arguments():
    from paper_2009_06404_amd import _lib as L
    for nu, tau, nk in ((0.5, 1.0, 17), (-0.1, 1.0, 17), (0.25, 0.5, 17), (0.25, 1.0, 1)):
        with pytest.raises(L.LBMError):
            L.lbm_vn_growth(nu, tau, nk)


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_2009_06404_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/liblbm.so")
    with pytest.raises(ImportError):
        L.lib()


def test_product_code_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2009_06404_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                with open(os.path.join(dirpath, f)) as fh:
                    text = fh.read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "lbm_oracle" not in text, f


@pytest.mark.parametrize("q,nu,tau", [(19, 0.25, 1.0), (19, 0.35, 1.0), (19, 0.1, 0.6), (27, 0.25, 1.0),
                                      (27, 0.37, 1.0), (27, 0.3, 0.55)])
def test_3d_stability_factor_matches_the_oracle_step(q, nu, tau):
    """lbm3_vn_growth (the library's own plane-wave step on D3Q19 / D3Q27,
    host code) on the wavenumbers {0, pi/2, pi}^3 against the largest
    eigenvalue modulus of the oracle's step matrix on those wavenumbers,
    read off one oracle step of plane waves on a periodic 4^3 volume."""
    import numpy as np
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_2009_06404_amd import _lib3d as L3
    from test_oracle_3d import _step_matrix
    from workloads.configs import lame_from_poisson
    lam, mu = lame_from_poisson(nu)
    best = 0.0
    for mx in range(3):
        for my in range(mx + 1):
            for mz in range(my + 1):
                M = _step_matrix((mx, my, mz), (4, 4, 4), lam, mu, tau, q)
                best = max(best, float(np.abs(np.linalg.eigvals(M)).max()))
    g = L3.lbm3_vn_growth(q, nu, tau, 3)
    assert abs(g - best) < 1e-7, (g, best)


def test_3d_stability_factor_window_and_arguments():
    from paper_2009_06404_amd import _lib as L
    from paper_2009_06404_amd import _lib3d as L3
    for q in (19, 27):
        assert L3.lbm3_vn_growth(q, 0.25, 1.0, 9) <= 1.0 + 1e-6     # nu = 1/4 is stable on both
        assert L3.lbm3_vn_growth(q, 0.37, 1.0, 9) > 1.01             # nu = 0.37 grows on both
    # D3Q19 grows from nu ~ 0.32 at tau = 1, where D3Q27 is still stable
    assert L3.lbm3_vn_growth(19, 0.33, 1.0, 9) > 1.01
    assert L3.lbm3_vn_growth(27, 0.33, 1.0, 9) <= 1.0 + 1e-6
    for args in ((15, 0.25, 1.0, 9), (19, 0.5, 1.0, 9), (19, 0.25, 0.5, 9), (19, 0.25, 1.0, 1)):
        with pytest.raises(L.LBMError):
            L3.lbm3_vn_growth(*args)
    import ctypes as C
    g = C.c_double(0)
    assert L3.lib().lbm3_stability(None, C.byref(g)) == L.LBM_E_INVALID
