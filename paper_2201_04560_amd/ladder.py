"""The mesh-refinement ladder of Sec. 3 on one GPU: per-mesh parameters of
the pool-boiling domain and a persistent cache of autotuned strip heights.

Mesh k has spacing dx = 2^-k of the base mesh and (base_nx 2^k) x
(base_ny 2^k) nodes.  a scales with dx^2 (Eq. a-deltax), T and the heater
temperature with T_c, sigma is refitted (Eq. integral_coexistence_curve),
kappa keeps gamma proportional to dx (Eq. gamma-meshes-relation), gravity
scales with dx^3 and the number of steps with dx^-2 (Table 1, viscous
regime); viscosities, c_v, conductivities, wall densities and all
relaxation rates are the same on every mesh."""
import json
import os
import tempfile

from .sim import make_params, refinement_level

B_EOS, OMEGA = 2.0 / 21.0, 0.344


def pool_level(k, a_base=2.0 / 49.0, Tr=0.86, T_heater_r=0.95, kappa0=0.0, gy0=-3e-5, steps0=100,
               base_nx=128, base_ny=256, heater_frac=0.125, rho_w=6.5, rho_w_heater=3.44,
               rho_w_top=0.38, cv=5.0, lambda_l=1.95, lambda_v=0.114, rates=None, precision=1,
               tile_y=0):
    """Parameters, wall columns and step count of mesh k of the pool-boiling
    ladder: heated strip of width heater_frac * nx centred on the bottom wall
    (Dirichlet T_heater_r T_c, wall density rho_w_heater), adiabatic
    elsewhere, top wall held at T_sat.  Returns a dict with 'params'
    (LbmParams), 'boundary' (keyword arguments of Lattice.set_boundary),
    'level' (the refinement_level record), 'nx', 'ny', 'steps'."""
    import numpy as np

    dx = 0.5 ** k
    lv = refinement_level(a_base, dx, Tr, kappa0, gy0, steps0, b=B_EOS, omega=OMEGA)
    nx, ny = base_nx * 2 ** k, base_ny * 2 ** k
    kw = dict(a=lv["a"], b=B_EOS, omega=OMEGA, sigma=lv["sigma"], kappa=lv["kappa"],
              rho_l=lv["rho_l"], rho_v=lv["rho_v"], walls=1, thermal=1, gy=lv["gy"], cv=cv,
              lambda_l=lambda_l, lambda_v=lambda_v, rho_ref=lv["rho_v"], precision=precision,
              tile_y=tile_y)
    if rates:
        kw.update(rates)
    p = make_params(nx, ny, **kw)
    hw = max(1, int(round(heater_frac * nx)))
    h0 = nx // 2 - hw // 2
    kind = np.full(nx, 2, np.int32)
    kind[h0:h0 + hw] = 1
    tb = np.full(nx, lv["T"])
    tb[h0:h0 + hw] = T_heater_r * lv["Tc"]
    rwb = np.full(nx, rho_w)
    rwb[h0:h0 + hw] = rho_w_heater
    bnd = dict(rho_w_bottom=rwb, rho_w_top=rho_w_top, t_bottom_kind=kind, t_bottom_val=tb,
               t_top_kind=1, t_top_val=lv["T"])
    return dict(params=p, boundary=bnd, level=lv, nx=nx, ny=ny, steps=int(lv["steps"]),
                heater=(h0, h0 + hw))


class TileCache:
    """Autotuned strip heights in a JSON file, keyed by lattice size,
    storage precision, wall and energy flags and the device name."""

    def __init__(self, path=None):
        self.path = path or os.environ.get(
            "LBM_PP_TILE_CACHE",
            os.path.join(os.path.expanduser("~"), ".cache", "paper_2201_04560_amd", "tile_y.json"))
        try:
            with open(self.path) as fh:
                self.table = json.load(fh)
        except (OSError, ValueError):
            self.table = {}

    @staticmethod
    def key(p, device=""):
        return (f"{p.nx}x{p.ny}/{'f32s' if p.precision else 'f64'}/walls{p.walls}/"
                f"thermal{p.thermal}/{device}")

    def lookup(self, p, device=""):
        """(tile_y, strip_waves) or None."""
        e = self.table.get(self.key(p, device))
        return None if e is None else (int(e["tile_y"]), int(e.get("strip_waves", 1)))

    def tune(self, lattice, candidates=(2, 3, 4, 5, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128), steps=20,
             device="", waves=(1, 2)):
        """Cached strip height and waves per strip for this lattice,
        autotuning (and storing) them on a miss; the lattice is set to them
        either way.  Returns (tile_y, strip_waves)."""
        hit = self.lookup(lattice.p, device)
        if hit is None:
            best = None
            for w in (waves if lattice.p.thermal else (1,)):
                lattice.strip_waves = w
                ty, ms = lattice.autotune_tile_y(candidates, steps)
                if best is None or ms < best[2]:
                    best = (ty, w, ms)
            hit = best[:2]
            self.table[self.key(lattice.p, device)] = {"tile_y": best[0], "strip_waves": best[1],
                                                       "ms_per_step": best[2],
                                                       "candidates": list(candidates)}
            self._save()
        lattice.tile_y, lattice.strip_waves = hit
        return hit

    def _save(self):
        d = os.path.dirname(self.path)
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
        with os.fdopen(fd, "w") as fh:
            json.dump(self.table, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
