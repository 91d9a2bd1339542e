"""CPU-only checks of the C-ABI library: it loads, exports every symbol of
include/lbm_pp.h, validates parameters and runs the host parameter
pipeline (compared with the independent oracle).  No GPU calls."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import thermo as th

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_pp.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2201_04560_amd import _native

    return _native.lib()


def test_every_declared_symbol_is_exported(lib):
    from paper_2201_04560_amd import _native

    names = header_functions()
    assert len(names) >= 20
    bound = {n for n, _, _ in _native.SIGNATURES}
    for n in names:
        assert hasattr(lib, n), n
        assert n in bound, f"{n} declared but not bound in Python"


def test_struct_sizes_match_header_layout(lib):
    from paper_2201_04560_amd._native import LbmNorms, LbmParams

    # 8 int32 + 22 double + 8 int32 + 8 double
    assert ctypes.sizeof(LbmParams) == 8 * 4 + 22 * 8 + 8 * 4 + 8 * 8
    assert ctypes.sizeof(LbmNorms) == 11 * 8 + 3 * 8


def test_validation(lib):
    from paper_2201_04560_amd import make_params
    from paper_2201_04560_amd._native import LBM_E_INVAL, LBM_OK

    ok = make_params(16, 16)
    assert lib.lbm_validate(ctypes.byref(ok)) == LBM_OK
    bad = [dict(nx=0), dict(ny=0), dict(a=0.0), dict(b=-1.0), dict(s_e=2.0), dict(s_q=0.0),
           dict(precision=7), dict(walls=1, ny=2), dict(thermal=1, cv=0.0), dict(tile_y=1),
           dict(rho_l=1.0, rho_v=1.0), dict(G=1.0), dict(n_iso=-1), dict(wall_model=2),
           dict(wall_model=-1), dict(strip_waves=3), dict(outflow_top=1), dict(outflow_top=2, walls=1)]
    for kw in bad:
        nx = kw.pop("nx", 16)
        ny = kw.pop("ny", 16)
        p = make_params(nx, ny, **kw)
        assert lib.lbm_validate(ctypes.byref(p)) == LBM_E_INVAL, kw
        n = ctypes.c_size_t()
        assert lib.lbm_buffer_bytes(ctypes.byref(p), ctypes.byref(n)) == LBM_E_INVAL
    assert lib.lbm_validate(None) == LBM_E_INVAL
    # an open top with gravity would need the outflow in the mean density
    p = make_params(16, 16, walls=1, outflow_top=1, gy=-1e-5)
    assert lib.lbm_validate(ctypes.byref(p)) == 6  # LBM_E_UNSUPPORTED
    p = make_params(16, 16, walls=1, outflow_top=1)
    assert lib.lbm_validate(ctypes.byref(p)) == LBM_OK


def test_buffer_bytes_cover_state(lib):
    from paper_2201_04560_amd import buffer_bytes, make_params

    for prec, elem in ((0, 8), (1, 4)):
        p = make_params(300, 200, precision=prec)
        n = buffer_bytes(p)
        assert n >= (2 * 9 + 2) * 300 * 200 * elem
        assert n < 1.5 * (2 * 9 + 2) * 320 * 200 * elem + (1 << 20)


def test_create_rejects_bad_buffers(lib):
    from paper_2201_04560_amd import make_params
    from paper_2201_04560_amd._native import LBM_E_INVAL, LBM_E_NOMEM

    p = make_params(16, 16)
    ctx = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(p), None, 1 << 20, None, ctypes.byref(ctx)) == LBM_E_INVAL
    assert lib.lbm_create(ctypes.byref(p), ctypes.c_void_p(256), 16, None,
                          ctypes.byref(ctx)) == LBM_E_NOMEM
    assert lib.lbm_create(ctypes.byref(p), ctypes.c_void_p(257), 1 << 30, None,
                          ctypes.byref(ctx)) == LBM_E_INVAL
    assert b"aligned" in lib.lbm_last_error(None)
    assert lib.lbm_status_string(5) == b"state left the EOS / pseudopotential domain"
    n = ctypes.c_int32()
    assert lib.lbm_tile_candidates(None, 0, None, 0, ctypes.byref(n)) == LBM_E_INVAL


@pytest.mark.parametrize("a", [2.0 / 49.0, 6.12e-2 * (128 / 288) ** 2])
def test_host_parameter_pipeline_matches_oracle(lib, a):
    import paper_2201_04560_amd as pp

    eos = th.EOS(a)
    assert abs(pp.pr_critical_temperature(a) - eos.Tc) < 1e-16
    T = 0.86 * eos.Tc
    rv, rl, ps = th.maxwell(eos, T)
    grv, grl, gps = pp.pr_maxwell(a, T)
    assert abs(grv - rv) < 1e-12 and abs(grl - rl) < 1e-11 and abs(gps - ps) < 1e-14
    s = th.fit_sigma(eos, T)
    assert abs(pp.fit_sigma(a, T) - s) < 1e-10
    g = th.planar_gamma_continuum(eos, T, s)
    assert abs(pp.planar_gamma(a, T, s) / g - 1) < 1e-7
    # Sec. 4.2: the library's closed-form h_fg against the oracle's quadrature
    h = th.latent_heat(eos, T, (rv, rl, ps))
    assert abs(pp.pr_latent_heat(a, T, rv, rl) / h - 1) < 1e-10


def test_stefan_beta_and_latent_heat_rejections(lib):
    """beta of Eq. stefan-analytical from the library against the oracle's
    bisection over the Jakob numbers of Sec. 4.2 and beyond; invalid inputs
    are refused."""
    import paper_2201_04560_amd as pp
    from paper_2201_04560_amd import LbmError

    for ja in (0.0, 1e-4, 0.038, 0.076, 0.133, 0.5, 3.0, 40.0):
        assert abs(pp.stefan_beta(ja) - th.stefan_beta(ja)) < 1e-12 * max(1.0, th.stefan_beta(ja))
    for bad in (-1e-3, float("nan"), float("inf")):
        with pytest.raises(LbmError):
            pp.stefan_beta(bad)
    a = 2.0 / 49.0
    T = 0.86 * pp.pr_critical_temperature(a)
    rv, rl, _ = pp.pr_maxwell(a, T)
    for args in ((a, T, rl, rv), (a, T, 0.0, rl), (a, 1.01 * T / 0.86, rv, rl), (a, T, rv, 11.0)):
        with pytest.raises(LbmError):
            pp.pr_latent_heat(*args)


def test_refinement_levels_match_oracle(lib):
    """Per-mesh a, Maxwell densities, sigma and kappa of the refinement
    ladder (Sec. 3) from the library against the oracle's independent
    implementation; the printed droplet meshes L = 128..432."""
    import paper_2201_04560_amd as pp

    a0 = 6.12e-3
    ref = th.refinement_parameters(a0, 128, [128, 192, 288, 432])
    for o in ref:
        lv = pp.refinement_level(a0, 128 / o["L"], gy0=-2.5e-5, steps0=400000)
        assert abs(lv["a"] / o["a"] - 1) < 1e-14
        assert abs(lv["rho_v"] - o["rho_v"]) < 1e-11 and abs(lv["rho_l"] - o["rho_l"]) < 1e-10
        assert abs(lv["sigma"] - o["sigma"]) < 1e-9
        assert abs(lv["kappa"] - o["kappa"]) < 1e-6, (o["L"], lv["kappa"], o["kappa"])
        assert abs(lv["gy"] / (-2.5e-5 * (128 / o["L"]) ** 3) - 1) < 1e-14
        assert lv["steps"] == round(400000 * (o["L"] / 128) ** 2)


def test_host_pipeline_rejects_supercritical(lib):
    import paper_2201_04560_amd as pp
    from paper_2201_04560_amd import LbmError

    with pytest.raises(LbmError):
        pp.pr_maxwell(2.0 / 49.0, 1.01 * pp.pr_critical_temperature(2.0 / 49.0))


def test_pool_ladder_levels(lib):
    """Mesh k of the ladder: 2^k times the base size, a ~ dx^2, g ~ dx^3,
    steps ~ dx^-2, heater strip an eighth of the width at 0.95 T_c(a_k)."""
    from paper_2201_04560_amd.ladder import pool_level

    base = pool_level(0, steps0=50)
    for k in range(4):
        L = pool_level(k, steps0=50)
        p, lv = L["params"], L["level"]
        assert (L["nx"], L["ny"]) == (128 * 2 ** k, 256 * 2 ** k) == (p.nx, p.ny)
        assert abs(p.a / base["params"].a - 4.0 ** -k) < 1e-15
        assert abs(p.gy / base["params"].gy - 8.0 ** -k) < 1e-14
        assert L["steps"] == 50 * 4 ** k
        h0, h1 = L["heater"]
        assert h1 - h0 == L["nx"] // 8
        tb = L["boundary"]["t_bottom_val"]
        assert abs(tb[h0] / lv["Tc"] - 0.95) < 1e-14 and abs(tb[0] / lv["Tc"] - 0.86) < 1e-14
        assert p.precision == 1 and p.walls == 1 and p.thermal == 1
        assert abs(p.rho_v - base["params"].rho_v) < 1e-10


def test_adjoint_bytes_and_scope(lib):
    import ctypes

    import paper_2201_04560_amd as pp

    p = pp.make_params(256, 256, thermal=1, precision=1)
    n1, n2 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lbm_adjoint_bytes(ctypes.byref(p), 500, 50, ctypes.byref(n1)) == 0
    assert lib.lbm_adjoint_bytes(ctypes.byref(p), 1000, 50, ctypes.byref(n2)) == 0
    assert n2.value > n1.value > 61 * 256 * 256 * 10 * 4  # 10 + 50 + 1 float32 states
    for kw in (dict(walls=1), dict(gy=-1e-5), dict(thermal=0)):
        q = pp.make_params(64, 64, **{**dict(thermal=1), **kw})
        assert lib.lbm_adjoint_bytes(ctypes.byref(q), 10, 5, ctypes.byref(n1)) == 6
    assert lib.lbm_adjoint_bytes(ctypes.byref(p), 0, 5, ctypes.byref(n1)) == 1


def test_droplet_refinement_meshes_match_table_2(lib):
    """Meshes of the Sec. 4.1 refinement from the product's rules: sigma
    reproduces Table 2's column, a scales with dx^2, the isothermal start
    with dx^-2, and the initial state has the Maxwell densities."""
    from paper_2201_04560_amd.ladder import droplet_mesh, droplet_radius

    printed_sigma = {128: 0.103, 192: 0.115, 288: 0.121, 432: 0.123}
    for L, s in printed_sigma.items():
        p, bnd, rho, T, lv = droplet_mesh(L)
        assert abs(p.sigma - s) <= 5e-4
        assert abs(p.a / 6.12e-2 - (128 / L) ** 2) < 1e-14
        assert p.n_iso == round(10000 * (L / 128) ** 2)
        assert abs(rho.max() - lv["rho_l"]) < 1e-6 and abs(rho.min() - lv["rho_v"]) < 1e-6
        assert abs(droplet_radius(rho, lv["rho_l"], lv["rho_v"]) - L / 4) < 0.05 * L / 4
