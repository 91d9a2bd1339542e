"""lbm_norms_device (the diagnostics for callers that cannot allocate) against
lbm_norms, through the C-ABI: two calls in a row on one GPU, the second on a
smaller lattice, each equal to lbm_norms on the same state."""
import ctypes

import numpy as np
import pytest

import cases

pytestmark = pytest.mark.gpu

_KEYS = ("mass", "rho_mean", "umax", "q_bottom", "q_heater", "l1_rho", "l2_rho", "linf_rho",
         "l1_T", "l2_T", "linf_T")


def _lattice(c, rho, T, precision, steps):
    from paper_2201_04560_amd import Lattice

    lat = Lattice(cases.lib_params(c, precision=precision))
    cases.lib_boundary(lat, c)
    lat.init_fields(rho, None, None, T)
    lat.step(steps)
    return lat


def _pool(nx, ny):
    eos, Tsat, rv, rl = cases.coexistence()
    kb = np.full(nx, 2)
    vb = np.full(nx, Tsat)
    h0, h1 = nx * 3 // 8, nx * 5 // 8
    kb[h0:h1] = 1
    vb[h0:h1] = 0.95 * eos.Tc
    c = dict(nx=nx, ny=ny, a=2.0 / 49.0, sigma=0.1103, kappa=0.0, rho_l=rl, rho_v=rv, walls=True,
             thermal=True, gy=-3e-5, cv=5.0, lambda_l=1.95, lambda_v=0.114,
             rho_w_bottom=np.where(kb == 1, 3.44, 6.5), rho_w_top=0.38, t_bottom_kind=kb,
             t_bottom_val=vb, t_top_kind=np.full(nx, 1), t_top_val=np.full(nx, Tsat),
             **cases.wl.POOL_RATES)
    rho, T = cases.wl.pool(nx, ny, ny * 0.6, 2.3, rl, rv, Tsat, seed_radius=5.0, seed=2)
    return c, rho, T


def _device_norms(lat):
    import torch

    from paper_2201_04560_amd._native import LbmNorms, check, lib

    out = torch.full((ctypes.sizeof(LbmNorms) // 8,), float("nan"), dtype=torch.float64,
                     device=lat._buf.device)
    check(lib().lbm_norms_device(lat._ctx, ctypes.c_void_p(out.data_ptr())), lat._ctx,
          "lbm_norms_device")
    host = out.cpu().numpy().copy()  # orders after the call on the current stream
    n = LbmNorms.from_buffer_copy(host.tobytes())
    return {k: getattr(n, k) for k, _ in LbmNorms._fields_}


@pytest.mark.parametrize("precision", [0, 1])
def test_norms_device_equals_norms_on_two_calls(precision):
    print(f"case norms_device precision={precision}: 96x64 pool then 40x24 pool", flush=True)
    big = _lattice(*_pool(96, 64), precision, 40)
    small = _lattice(*_pool(40, 24), precision, 25)
    for lat in (big, small):
        d = _device_norms(lat)
        h = lat.norms()
        print({k: f"{abs(d[k] - h[k]) / max(abs(h[k]), 1e-300):.1e}" for k in _KEYS}, flush=True)
        for k in _KEYS:
            assert abs(d[k] - h[k]) <= 1e-15 * max(abs(h[k]), 1e-300), (k, d[k], h[k])
        for k in ("nonfinite", "n_heater", "step"):
            assert d[k] == h[k], (k, d[k], h[k])
        assert d["n_heater"] == lat.nx // 4 and d["q_heater"] != 0.0
    # the second call left the small lattice's sums in the shared array; a
    # third call on the big lattice again matches
    d = _device_norms(big)
    h = big.norms()
    for k in _KEYS:
        assert abs(d[k] - h[k]) <= 1e-15 * max(abs(h[k]), 1e-300), (k, d[k], h[k])
    big.close()
    small.close()
