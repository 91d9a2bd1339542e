"""Laplace law (Eq. laplace-equation, Sec. 3.1) on static droplets of the
oracle, and the surface-tension law gamma(kappa) = (1 - kappa) gamma(0) of
Eq. surface_tension (Sec. 3.2).

Measurement (the standard static-droplet procedure): a liquid disk of
radius R0 relaxes on an n x n periodic lattice (config-1 parameters:
a = 2/49, T = 0.86 T_c, sigma = 0.1, all rates 1.25); at the end
  rho_in  = mean density of the 2 x 2 centre nodes,
  rho_out = density at the corner (0, 0), far from the droplet,
  R       = equimolar radius, pi R^2 = (sum rho - N rho_out) / (rho_in - rho_out),
  dp      = p_EOS(rho_in) - p_EOS(rho_out).
On a periodic lattice the droplet gives up mass to the vapour until the
vapour is supersaturated to the Kelvin value, so R is measured from the
final bulk densities, not from the initial radius or a liquid fraction
clipped between the coexistence densities (that sum is fixed by the
conserved total mass).  gamma is the slope of dp against 1/R.

Run as a script, it performs the full study (R0 = 15 ... 35 on 128^2,
20,000 steps, kappa = 0, 0.1, 0.3, -0.2) with the oracle and writes
laplace_128.json next to this file, with the sha256 of the oracle sources
it ran on.  Test infrastructure: calls only oracle/ and workloads/.
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import thermo as th  # noqa: E402
from oracle.step import Params, Sim  # noqa: E402

import workloads as wl  # noqa: E402

A = 2.0 / 49.0
EOS = th.EOS(A)
T86 = 0.86 * EOS.Tc
SIGMA = 0.1
ORACLE_FILES = ["oracle/__init__.py", "oracle/lattice.py", "oracle/step.py", "oracle/thermo.py"]


def oracle_sha256():
    h = hashlib.sha256()
    for f in ORACLE_FILES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def droplet_point(args):
    """(R, dp) of one static droplet: args = (kappa, R0, n, steps)."""
    kappa, r0, n, steps = args
    rv, rl, _ = th.coexistence_for_sigma(EOS, T86, SIGMA)
    rho, T = wl.droplet(n, n, r0, 4.6 / 2.0, rl, rv, T86, T86)
    s = Sim(Params(nx=n, ny=n, a=A, sigma=SIGMA, kappa=kappa, rho_l=rl, rho_v=rv))
    s.init_fields(rho, T=T)
    s.step(steps)
    r = s.fields()[0]
    c = n // 2
    rin = float(r[c - 1:c + 1, c - 1:c + 1].mean())
    rout = float(r[0, 0])
    R = float(np.sqrt((r.sum() - r.size * rout) / (rin - rout) / np.pi))
    dp = float(EOS.p(rin, T86) - EOS.p(rout, T86))
    return R, dp


def fit(points):
    """gamma (slope of dp vs 1/R), intercept, R^2 of the linear fit."""
    X = np.array([1.0 / R for R, _ in points])
    Y = np.array([d for _, d in points])
    slope, icpt = np.polyfit(X, Y, 1)
    r2 = 1.0 - ((Y - (slope * X + icpt)) ** 2).sum() / ((Y - Y.mean()) ** 2).sum()
    return float(slope), float(icpt), float(r2), float(Y.max() - Y.min())


def study(n, steps, radii, kappas, workers=None):
    """gamma for each kappa from droplets of the given radii (a process pool
    over the independent droplets)."""
    from multiprocessing import Pool

    jobs = [(k, r, n, steps) for k in kappas for r in radii]
    workers = workers or min(len(jobs), max(1, (os.cpu_count() or 1)))
    with Pool(workers) as pool:
        pts = pool.map(droplet_point, jobs)
    out = {}
    for k in kappas:
        p = [pt for (kk, *_), pt in zip(jobs, pts) if kk == k]
        g, icpt, r2, rng = fit(p)
        out[k] = dict(gamma=g, intercept=icpt, r2=r2, dp_range=rng, points=p)
    return out


if __name__ == "__main__":
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    radii, kappas, n, steps = [15.0, 20.0, 25.0, 30.0, 35.0], [0.0, 0.1, 0.3, -0.2], 128, 20000
    res = study(n, steps, radii, kappas)
    doc = {"what": "static droplets of the oracle: gamma = slope of dp against 1/R per kappa",
           "n": n, "steps": steps, "radii": radii, "sigma": SIGMA, "T_over_Tc": 0.86, "a": A,
           "planar_gamma_continuum_kappa0": th.planar_gamma_continuum(EOS, T86, SIGMA, 0.0),
           "oracle_sha256": oracle_sha256(), "script": "tests/golden/laplace_study.py",
           "kappa": {str(k): v for k, v in res.items()}}
    with open(os.path.join(HERE, "laplace_128.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")
    for k, v in res.items():
        print(f"kappa {k:+.2f}: gamma {v['gamma']:.5e} R2 {v['r2']:.6f} "
              f"intercept/range {v['intercept'] / v['dp_range']:+.4f}")
