"""Seeded synthetic workloads: initial fields and parameter recipes.

This module holds no arithmetic of the method (no EOS, no forces, no
collision): it only draws seeded random numbers and lays out initial
density / temperature fields of given phase values.  It is shared by the
test suite, the benchmark and the smoke check; the GPU library and the
oracle receive its arrays as plain inputs.

Random numbers: splitmix64 (Steele, Lea, Flood 2014) of seed * 2^32 +
node index, converted to a double in [0, 1) from the top 53 bits.

Workloads (physical setups of Sec. 4 of the paper, in lattice units):
  droplet  -- a liquid disk in vapour with the tanh profile of Sec. 4.1;
              liquid inside (the printed sign puts the vapour inside, read
              as a sign slip), width parameter k = 4.6 / W
  pool     -- liquid below a height, vapour above (Sec. 4.3), smoothed
              by the same tanh profile, with a vapour half-disk nucleation
              site centred on the bottom wall
Recipes for the five benchmark configurations are the dicts below.
"""
import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """splitmix64 finaliser applied to uint64 array x (wrapping arithmetic)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, idx):
    """Counter-based uniform doubles in [0, 1) for node indices idx."""
    key = (np.uint64(seed) << np.uint64(32)) + np.asarray(idx, dtype=np.uint64)
    z = splitmix64(key)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def jitter(seed, nx, ny, amplitude=0.5):
    """Per-node offsets in [-amplitude, amplitude), shape [ny, nx]."""
    if seed is None:
        return np.zeros((ny, nx))
    idx = np.arange(nx * ny, dtype=np.uint64).reshape(ny, nx)
    return (2.0 * uniform01(seed, idx) - 1.0) * amplitude


def tanh_blend(d, r0, k, inside, outside):
    """inside for d << r0, outside for d >> r0, tanh of width 1/k between."""
    return 0.5 * (inside + outside) - 0.5 * (inside - outside) * np.tanh(k * (d - r0))


def droplet(nx, ny, r0, k, rho_in, rho_out, T_in, T_out, centre=None, seed=None,
            amplitude=0.5):
    """Liquid disk of radius r0 (+ seeded per-node jitter) centred in the box.
    Returns (rho, T) arrays of shape [ny, nx]."""
    cx, cy = (nx / 2.0, ny / 2.0) if centre is None else centre
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    r = r0 + jitter(seed, nx, ny, amplitude)
    rho = tanh_blend(d, r, k, rho_in, rho_out)
    T = tanh_blend(d, r, k, T_in, T_out)
    return rho, T


def pool(nx, ny, height, k, rho_l, rho_v, T0, seed_radius=8.0, seed=None, amplitude=0.5):
    """Liquid for y < height, vapour above, plus a vapour half-disk of radius
    seed_radius (+ jitter) centred at (nx/2, 0).  Returns (rho, T)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    j = jitter(seed, nx, ny, amplitude)
    rho = tanh_blend(y, height, k, rho_l, rho_v)
    if seed_radius > 0:
        d = np.sqrt((x - nx / 2.0) ** 2 + y**2)
        bub = tanh_blend(d, seed_radius + j, k, 1.0, 0.0)  # 1 inside the nucleus
        rho = rho * (1.0 - bub) + rho_v * bub
    T = np.full((ny, nx), float(T0))
    return rho, T


# ---------------------------------------------------------------------------
# recipes: numbers only; T_r is relative to T_c(a), densities are the
# coexistence densities of the EOS at T_r (computed by the caller)
# ---------------------------------------------------------------------------
DROPLET_RATES = dict(s_rho=1.25, s_e=1.25, s_zeta=1.25, s_j=1.25, s_q=1.25)  # Sec. 4.1
POOL_RATES = dict(s_rho=1.0, s_e=0.8, s_zeta=0.8, s_j=1.0, s_q=1.1)  # Sec. 4.2/4.3

CONFIGS = {
    # plain FP64 static droplet, isothermal
    "droplet128": dict(nx=128, ny=128, a=2.0 / 49.0, Tr=0.86, r0=25.0, width=2.0,
                       sigma=0.1, kappa=0.1, steps=1000, thermal=False, seed=None,
                       **DROPLET_RATES),
    # droplet vaporisation: liquid at T_sat in vapour held at 0.95 T_c
    "droplet512": dict(nx=512, ny=512, a=2.0 / 49.0, Tr=0.86, Tr_out=0.95, r0=60.0,
                       width=5.0, sigma=0.1, kappa=0.1, cv=6.0, lam=2.0 / 3.0,
                       steps=20000, thermal=True, seed=0, **DROPLET_RATES),
    # pool boiling, 1024 wide x 2048 tall
    "pool1024x2048": dict(nx=1024, ny=2048, a=2.0 / 49.0, Tr=0.86, Tr_heater=0.95,
                          height=1400.0, width=2.0, gy=-3e-5, heater=(448, 576),
                          sigma=0.1103, kappa=0.0, cv=5.0, lambda_l=1.95, lambda_v=0.114,
                          rho_w_top=0.38, rho_w_bottom=6.50, rho_w_heater=0.38,
                          steps=50000, thermal=True, seed=0, **POOL_RATES),
    # adjoint: 256^2 droplet vaporisation, bottom row is the control
    "adjoint256": dict(nx=256, ny=256, a=2.0 / 49.0, Tr=0.86, Tr_out=0.95, r0=30.0,
                       width=5.0, sigma=0.1, kappa=0.1, cv=6.0, lam=2.0 / 3.0,
                       steps=500, checkpoint=50, thermal=True, seed=0, **DROPLET_RATES),
}
