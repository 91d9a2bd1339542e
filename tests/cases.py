"""Shared test cases: one plain dict of numbers per case, turned into the
oracle's Params and the library's LbmParams by two independent adapters
(the oracle side never imports the library and vice versa)."""
import numpy as np

import workloads as wl
from oracle import thermo as th
from oracle.step import Params

T_FREE, T_DIRICHLET, T_ADIABATIC = 0, 1, 2


def oracle_params(c):
    keys = ["nx", "ny", "a", "sigma", "kappa", "s_rho", "s_e", "s_zeta", "s_j", "s_q", "eta_l",
            "eta_v", "rho_l", "rho_v", "gy", "walls", "thermal", "n_iso", "cv", "lambda_l",
            "lambda_v", "rho_w_bottom", "rho_w_top", "t_bottom_kind", "t_bottom_val", "t_top_kind",
            "t_top_val", "t_side_dirichlet", "t_side_val", "wall_model", "gw_bottom", "gw_top",
            "outflow_top"]
    return Params(**{k: c[k] for k in keys if k in c})


def lib_params(c, precision=0, tile_y=0, rho_ref=None, xcd_remap=1, strip_waves=0):
    from paper_2201_04560_amd import make_params

    scal = ["a", "sigma", "kappa", "s_rho", "s_e", "s_zeta", "s_j", "s_q", "eta_l", "eta_v",
            "rho_l", "rho_v", "gy", "cv", "lambda_l", "lambda_v", "t_side_val"]
    kw = {k: float(c[k]) for k in scal if k in c}
    for k in ("walls", "thermal", "n_iso", "t_side_dirichlet", "wall_model", "outflow_top"):
        if k in c:
            kw[k] = int(c[k])
    kw["precision"] = precision
    kw["tile_y"] = tile_y
    kw["xcd_remap"] = xcd_remap
    kw["strip_waves"] = strip_waves
    kw["rho_ref"] = float(c.get("rho_v", 0.38) if rho_ref is None else rho_ref)
    return make_params(c["nx"], c["ny"], **kw)


def lib_boundary(lat, c):
    nx = c["nx"]
    col = lambda k, d: np.broadcast_to(np.asarray(c.get(k, d)), (nx,))
    # the wall tables hold rho_w (psi-based) or G_w (modified-psi walls)
    wb, wt = ("gw_bottom", "gw_top") if c.get("wall_model", 0) == 1 else ("rho_w_bottom", "rho_w_top")
    dflt = -1.0 if c.get("wall_model", 0) == 1 else 1.0
    lat.set_boundary(col(wb, dflt), col(wt, dflt),
                     col("t_bottom_kind", 0).astype(np.int32), col("t_bottom_val", 0.0),
                     col("t_top_kind", 0).astype(np.int32), col("t_top_val", 0.0))


def coexistence(a=2.0 / 49.0, tr=0.86):
    eos = th.EOS(a)
    T = tr * eos.Tc
    rv, rl, _ = th.maxwell(eos, T)
    return eos, T, rv, rl


def droplet128():
    """Plain FP64 static droplet, 128^2 periodic, isothermal (1000 steps)."""
    eos, T, rv, rl = coexistence()
    c = dict(nx=128, ny=128, a=2.0 / 49.0, sigma=0.1, kappa=0.1, rho_l=rl, rho_v=rv,
             **wl.DROPLET_RATES)
    rho, Tf = wl.droplet(128, 128, 25.0, 4.6 / 2.0, rl, rv, T, T)
    return c, rho, Tf


def random_tiny(nx, ny, seed, walls=False, thermal=False, gy=0.0, wall_model=0, outflow_top=False):
    """Random near-equilibrium state inside the EOS domain, exercising every
    term: walls with random wall densities (or random G_w for modified-psi
    walls), mixed temperature kinds."""
    eos, T, rv, rl = coexistence()
    rng = np.random.default_rng(seed)
    c = dict(nx=nx, ny=ny, a=2.0 / 49.0, sigma=0.11, kappa=0.3, rho_l=rl, rho_v=rv,
             s_rho=1.0, s_e=0.8, s_zeta=0.9, s_j=1.1, s_q=1.3, eta_l=0.15, eta_v=0.07,
             gy=gy, walls=walls, thermal=thermal, cv=5.0, lambda_l=0.9, lambda_v=0.2)
    if walls:
        c["rho_w_bottom"] = rng.uniform(0.5, 6.0, nx)
        c["rho_w_top"] = rng.uniform(0.5, 6.0, nx)
        if outflow_top:
            c["outflow_top"] = True
        if wall_model == 1:
            c["wall_model"] = 1
            c["gw_bottom"] = rng.uniform(-1.4, -0.6, nx)
            c["gw_top"] = rng.uniform(-1.4, -0.6, nx)
        kb = rng.integers(1, 3, nx)
        kt = rng.integers(1, 3, nx)
        c["t_bottom_kind"], c["t_top_kind"] = kb, kt
        c["t_bottom_val"] = rng.uniform(0.87, 0.95, nx) * eos.Tc
        c["t_top_val"] = rng.uniform(0.87, 0.95, nx) * eos.Tc
    rho = rng.uniform(0.45, 6.2, (ny, nx))
    ux = rng.uniform(-0.02, 0.02, (ny, nx))
    uy = rng.uniform(-0.02, 0.02, (ny, nx))
    Tf = rng.uniform(0.85, 0.93, (ny, nx)) * eos.Tc
    return c, rho, ux, uy, Tf


def heater_case(nx=16, ny=14, r=3.5, cy=5.0, seed=3, k=1.2):
    """Droplet vaporisation inside a Dirichlet ring whose bottom row (the
    heater profile) varies by +-1 % around 0.95 T_c; the droplet sits near
    the heater.  Returns (case dict, rho, T, rho_mid, width)."""
    eos, Tsat, rv, rl = coexistence()
    Tout = 0.95 * eos.Tc
    rng = np.random.default_rng(seed)
    tb = Tout * (1.0 + 0.01 * rng.uniform(-1, 1, nx))
    c = dict(nx=nx, ny=ny, a=2.0 / 49.0, sigma=0.1, kappa=0.1, rho_l=rl, rho_v=rv, thermal=True,
             cv=6.0, lambda_l=2 / 3, lambda_v=2 / 3, t_side_dirichlet=True, t_side_val=Tout,
             t_bottom_kind=np.full(nx, T_DIRICHLET), t_bottom_val=tb,
             t_top_kind=np.full(nx, T_DIRICHLET), t_top_val=np.full(nx, Tout), **wl.DROPLET_RATES)
    rho, T = wl.droplet(nx, ny, r, k, rl, rv, Tsat, Tout, centre=(nx / 2, cy), seed=seed)
    return c, rho, T, 0.5 * (rl + rv), (rl - rv) / 8.0
