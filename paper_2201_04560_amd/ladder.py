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

from .sim import make_params, refinement_level, stefan_beta
from .sim import pr_latent_heat as _pr_latent_heat

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
            best, tried = None, set()
            for w in (waves if lattice.p.thermal else (1,)):
                lattice.strip_waves = w
                # the fixed ladder plus the heights that fill whole rounds of
                # wave slots (a launch a few waves over such a round leaves
                # some SIMDs with one wave more: 4096^2 float32 pool 128 rows
                # -> 514 us, 100 rows -> 433 us on MI355X)
                cand = sorted(set(candidates) | set(lattice.tile_candidates(w)))
                tried.update(cand)
                ty, ms = lattice.autotune_tile_y(cand, steps)
                if best is None or ms < best[2]:
                    best = (ty, w, ms)
            hit = best[:2]
            self.table[self.key(lattice.p, device)] = {"tile_y": best[0], "strip_waves": best[1],
                                                       "ms_per_step": best[2],
                                                       "candidates": sorted(tried)}
            self._save()
        lattice.tile_y, lattice.strip_waves = hit
        return hit

    def tune_batch(self, make_lattices, device="",
                   candidates=(4, 6, 8, 12, 13, 16, 20, 24, 26, 32, 40, 48, 52, 64, 80, 96, 128),
                   steps=10, waves=(1,), with_waves=False):
        """Strip height (and waves per strip) for same-shaped lattices
        advanced together by one batched launch.  A batch holds n times the
        workgroups of one lattice, so it can afford taller strips (fewer
        recomputed halo rows) than the lattice alone.  On a miss, times the
        batched launch for each candidate height and each entry of `waves`
        (2: the two-wave march, energy-equation lattices) on throwaway
        lattices from make_lattices() (initialised, same shape) and caches the
        fastest under the lattice key + "/batch<n>" (+ "w12" when two waves
        were tried).  Returns the height, or (height, waves) with
        with_waves=True."""
        lats = None
        key = None
        e = None
        try:
            lats = make_lattices()
            n = len(lats)
            ws = tuple(w for w in waves if w == 1 or lats[0].p.thermal)
            tag = "" if ws == (1,) else "w" + "".join(str(w) for w in ws)
            key = self.key(lats[0].p, f"{device}/batch{n}{tag}")
            e = self.table.get(key)
            if e is None:
                from .sim import Batch

                best, tried = None, []
                for w in ws:
                    for ty in candidates:
                        if ty > max(lats[0].ny, 2):
                            continue
                        for lat in lats:
                            lat.tile_y = ty
                            lat.strip_waves = w
                        b = Batch(lats)
                        try:
                            b.run([2] * n)
                            b.run([steps] * n)
                            ms = b.last_time()[0] / steps
                        finally:
                            b.close()
                        tried.append([ty, w])
                        if best is None or ms < best[2]:
                            best = (ty, w, ms)
                e = {"tile_y": best[0], "strip_waves": best[1], "ms_per_step": best[2],
                     "candidates": tried}
                self.table[key] = e
                self._save()
        finally:
            for lat in lats or []:
                lat.close()
        if with_waves:
            return int(e["tile_y"]), int(e.get("strip_waves", 1))
        return int(e["tile_y"])

    def _save(self):
        d = os.path.dirname(self.path)
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
        with os.fdopen(fd, "w") as fh:
            json.dump(self.table, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


# ----------------------------------------------------------------------------
# droplet-vaporisation refinement study (Secs. 3 and 4.1)
# ----------------------------------------------------------------------------
def droplet_radius(rho, rho_l, rho_v):
    """R = sqrt(A / pi) with A the liquid area: the smooth indicator
    H = (1 + tanh((rho - rho_mid) / w)) / 2, rho_mid = (rho_l + rho_v) / 2,
    w = (rho_l - rho_v) / 8, summed over the nodes.  (A clipped liquid
    fraction (rho - rho_v) / (rho_l - rho_v) would sum to the total mass on a
    periodic lattice, which the scheme conserves, and miss the interface.)"""
    import numpy as np

    mid, w = 0.5 * (rho_l + rho_v), (rho_l - rho_v) / 8.0
    return float(np.sqrt((0.5 * (1.0 + np.tanh((rho - mid) / w))).sum() / np.pi))


def droplet_mesh(L, L0=128, a0=6.12e-2, R0_frac=0.25, Tr=0.86, Tv_r=1.0, iso0=10000, cv=5.0,
                 lam=2.0 / 3.0, eta=0.1, precision=0, tile_y=0):
    """Mesh L of the droplet-vaporisation refinement (Sec. 4.1): L x L
    periodic lattice, liquid disk of radius R0_frac L at T_sat = Tr T_c in
    vapour at Tv_r T_c, temperature ring held at the vapour value; a, sigma,
    kappa from the refinement rule with dx = L0 / L; the energy equation
    starts after iso0 (L / L0)^2 steps.  Returns (params, boundary, rho, T,
    level record)."""
    import numpy as np

    from .sim import make_params, refinement_level

    dx = L0 / L
    lv = refinement_level(a0, dx, Tr)
    Tc, Ts = lv["Tc"], lv["T"]
    Tv = Tv_r * Tc
    rates = dict(s_rho=1.25, s_e=1.25, s_zeta=1.25, s_j=1.25, s_q=1.25)
    p = make_params(L, L, a=lv["a"], sigma=lv["sigma"], kappa=lv["kappa"], rho_l=lv["rho_l"],
                    rho_v=lv["rho_v"], thermal=1, n_iso=int(round(iso0 / dx ** 2)), cv=cv,
                    lambda_l=lam, lambda_v=lam, eta_l=eta, eta_v=eta, t_side_dirichlet=1,
                    t_side_val=Tv, rho_ref=lv["rho_v"], precision=precision, tile_y=tile_y, **rates)
    bnd = dict(t_bottom_kind=np.full(L, 1, np.int32), t_bottom_val=np.full(L, Tv),
               t_top_kind=np.full(L, 1, np.int32), t_top_val=np.full(L, Tv))
    y, x = np.mgrid[0:L, 0:L].astype(np.float64)
    d = np.hypot(x - L / 2 + 0.5, y - L / 2 + 0.5)
    # Sec. 4.1 initial profile, width 4.6/5.0 on the base mesh (scaled with it)
    t = np.tanh((4.6 / 5.0) * dx * (d - R0_frac * L))
    rho = 0.5 * (lv["rho_v"] + lv["rho_l"]) - 0.5 * (lv["rho_l"] - lv["rho_v"]) * t
    T = 0.5 * (Tv + Ts) - 0.5 * (Ts - Tv) * t
    return p, bnd, rho, T, lv


def droplet_refinement(meshes=(128, 192, 288, 432), L0=128, samples=200, sample0=2048,
                       precision=0, progress=None, **kw):
    """Run every mesh of the refinement in one batch (one multi-lattice
    launch per step, graph-replayed), mesh L advanced sample0 (L / L0)^2
    steps between samples of the droplet radius (the same physical times on
    every mesh, Delta t ~ Delta x^2).  Returns the radius histories in base
    mesh units, Delta*R between consecutive meshes (Eq. relative-change-R)
    and the convergence orders log(Delta*_k / Delta*_k+1) / log(ratio)."""
    import math

    import numpy as np

    from .sim import Batch, Lattice

    lats, steps, levels = [], [], []
    for L in meshes:
        s = sample0 * (L / L0) ** 2
        if abs(s - round(s)) > 1e-9:
            raise ValueError("sample0 (L / L0)^2 must be an integer for every mesh")
        p, bnd, rho, T, lv = droplet_mesh(L, L0, precision=precision, **kw)
        lat = Lattice(p)
        lat.set_boundary(**bnd)
        lat.init_fields(rho, None, None, T)
        lats.append(lat)
        steps.append(int(round(s)))
        levels.append(lv)
    R = np.zeros((len(meshes), samples + 1))
    for m, (lat, lv) in enumerate(zip(lats, levels)):
        R[m, 0] = droplet_radius(lat.fields()[0], lv["rho_l"], lv["rho_v"]) * L0 / meshes[m]
    b = Batch(lats)
    for k in range(1, samples + 1):
        b.run(steps)
        for m, (lat, lv) in enumerate(zip(lats, levels)):
            R[m, k] = droplet_radius(lat.fields()[0], lv["rho_l"], lv["rho_v"]) * L0 / meshes[m]
        if progress:
            progress(k, samples)
    b.close()
    for lat in lats:
        lat.close()
    dstar = [float(np.abs(R[m] - R[m + 1]).sum() / np.abs(R[m + 1]).sum())
             for m in range(len(meshes) - 1)]
    ratio = meshes[1] / meshes[0]
    orders = [math.log(dstar[m] / dstar[m + 1]) / math.log(ratio) for m in range(len(dstar) - 1)]
    return {"meshes": list(meshes), "steps_per_sample": steps, "samples": samples, "R": R,
            "delta_star_R": dstar, "orders": orders,
            "kappa": [lv["kappa"] for lv in levels], "sigma": [lv["sigma"] for lv in levels],
            "a": [lv["a"] for lv in levels]}


# ----------------------------------------------------------------------------
# pool-boiling refinement: space / space-time differences between meshes
# and the time-shift synchronisation (Sec. 4.3)
# ----------------------------------------------------------------------------
def pool_mesh(N, N0=160, a0=6.12e-2, Tr=0.86, Th_r=1.0, rho_wh=3.44, heater_frac=0.05,
              gy0=-2.5e-5, cv=5.0, lambda_l=1.95, lambda_v=0.114, eta=0.1, precision=0, tile_y=0):
    """Mesh N (N x N) of the Sec. 4.3 pool: periodic sides, Zou-He walls,
    liquid below half the height at T_sat = Tr T_c, top wall at T_sat with
    wall density 0.38, bottom wall at T_sat with wall density 6.50 except the
    centred heater (heater_frac N nodes) at Th_r T_c with density rho_wh;
    a, sigma, kappa and g by the refinement rules with dx = N0 / N.
    Returns (params, boundary, rho, T, level record)."""
    import numpy as np

    from .sim import make_params, refinement_level

    dx = N0 / N
    lv = refinement_level(a0, dx, Tr, 0.0, gy0)
    Tc, Ts = lv["Tc"], lv["T"]
    rates = dict(s_rho=1.0, s_e=0.8, s_zeta=0.8, s_j=1.0, s_q=1.1)
    p = make_params(N, N, a=lv["a"], sigma=lv["sigma"], kappa=lv["kappa"], rho_l=lv["rho_l"],
                    rho_v=lv["rho_v"], walls=1, thermal=1, gy=lv["gy"], cv=cv, lambda_l=lambda_l,
                    lambda_v=lambda_v, eta_l=eta, eta_v=eta, rho_ref=lv["rho_v"],
                    precision=precision, tile_y=tile_y, **rates)
    hw = max(1, int(round(heater_frac * N)))
    h0 = N // 2 - hw // 2
    tb = np.full(N, Ts)
    tb[h0:h0 + hw] = Th_r * Tc
    rwb = np.full(N, 6.50)
    rwb[h0:h0 + hw] = rho_wh
    bnd = dict(rho_w_bottom=rwb, rho_w_top=0.38, t_bottom_kind=np.full(N, 1, np.int32),
               t_bottom_val=tb, t_top_kind=np.full(N, 1, np.int32), t_top_val=Ts)
    y = (np.arange(N, dtype=np.float64)[:, None] + 0.5) * np.ones((1, N))
    # Eq. boundary-cond: liquid below half the height (smoothed over one
    # base-mesh node)
    t = np.tanh((y - N / 2) * dx)
    rho = 0.5 * (lv["rho_l"] + lv["rho_v"]) - 0.5 * (lv["rho_l"] - lv["rho_v"]) * t
    T = np.full((N, N), Ts)
    return p, bnd, rho, T, lv


def bilinear(coarse, n_fine, periodic_x=True):
    """Coarse node-centred field [Nc, Nc'] interpolated linearly onto the
    node centres of the fine mesh [n_fine, n_fine'] covering the same domain
    (periodic in x, clamped in y)."""
    import numpy as np

    ncy, ncx = coarse.shape
    nfy, nfx = (n_fine, n_fine) if np.isscalar(n_fine) else n_fine
    yc = (np.arange(nfy) + 0.5) * ncy / nfy - 0.5
    xc = (np.arange(nfx) + 0.5) * ncx / nfx - 0.5
    yc = np.clip(yc, 0.0, ncy - 1.0)
    y0 = np.minimum(np.floor(yc).astype(int), ncy - 2)
    fy = yc - y0
    x0 = np.floor(xc).astype(int)
    fx = xc - x0
    xa, xb = x0 % ncx, (x0 + 1) % ncx
    if not periodic_x:
        xa, xb = np.clip(x0, 0, ncx - 1), np.clip(x0 + 1, 0, ncx - 1)
    c = coarse
    top = c[y0][:, xa] * (1 - fx) + c[y0][:, xb] * fx
    bot = c[y0 + 1][:, xa] * (1 - fx) + c[y0 + 1][:, xb] * fx
    return top * (1 - fy)[:, None] + bot * fy[:, None]


def space_difference(coarse, fine):
    """Eq. rel-diff-timestep: sum |I(coarse) - fine| / sum |fine|."""
    import numpy as np

    i = bilinear(coarse, fine.shape)
    return float(np.abs(i - fine).sum() / np.abs(fine).sum())


def best_shift(series_coarse, fine_ref, shifts):
    """Eq. rel-diff-minimize: the shift whose coarse field (interpolated)
    differs least, in L1, from the finest field at the reference time.
    series_coarse maps shift -> field."""
    import numpy as np

    best, arg = None, None
    for d in shifts:
        v = np.abs(bilinear(series_coarse[d], fine_ref.shape) - fine_ref).sum()
        if best is None or v < best:
            best, arg = v, d
    return arg


def pool_refinement(meshes=(160, 240, 360, 540), N0=160, steps0=40000, every0=640, tau0=5120,
                    m0=4800, shift_every0=320, precision=0, progress=None, **kw):
    """Sec. 4.3 study, every mesh in one batch.  Pass 1 samples rho and T
    every every0 base-mesh steps (the same physical times on every mesh)
    and every shift_every0 steps in [tau0 - m0, tau0 + m0]; it gives the
    space differences d^N(t) of rho and T between consecutive meshes
    (Eq. rel-diff-timestep), the global differences D^N (Eq.
    global-rel-diff) with their convergence orders, and the time shift
    delta of every coarser mesh against the finest at tau0 (Eq.
    rel-diff-minimize).  Pass 2 reruns the coarser meshes with a non-zero
    shift and samples them at the shifted times t_k (1 + delta / tau0),
    rounded to whole steps of each mesh, for the shifted global differences
    (Eq. global-rel-diff-shifted).  Also returned: the heat flux Q(t) of
    Eq. pool-heat-flux per mesh (re-scaled to the base mesh), the relative
    differences of consecutive Q curves over t > 0 and their orders, and
    the vapour area under the initial interface (bubble growth and
    departure)."""
    import math

    import numpy as np

    from .sim import Batch, Lattice

    ratios = [(N / N0) ** 2 for N in meshes]  # steps of mesh N per base step
    for v in (steps0, every0, tau0, m0, shift_every0):
        for N, q in zip(meshes, ratios):
            if abs(v * q - round(v * q)) > 1e-9:
                raise ValueError(f"{v} base steps are not a whole number of steps on mesh {N}")
    if tau0 + m0 > steps0 or tau0 - m0 < 0:
        raise ValueError("the shift window must lie inside the run")
    nm = len(meshes)

    def build(idx):
        lats, levels = [], []
        for m in idx:
            p, bnd, rho, T, lv = pool_mesh(meshes[m], N0, precision=precision, **kw)
            lat = Lattice(p)
            lat.set_boundary(**bnd)
            lat.init_fields(rho, None, None, T)
            lats.append(lat)
            levels.append(lv)
        return lats, levels

    def march(idx, targets, take, label):
        """Advance meshes idx through the per-mesh step counts targets[j]
        (one row per event) and call take(j, event, lattice, level) at each."""
        lats, levels = build(idx)
        for j, (lat, lv) in enumerate(zip(lats, levels)):
            take(j, 0, lat, lv)
        b = Batch(lats)
        done = [0] * len(idx)
        for e in range(1, len(targets)):
            b.run([targets[e][j] - done[j] for j in range(len(idx))])
            done = list(targets[e])
            for j, (lat, lv) in enumerate(zip(lats, levels)):
                take(j, e, lat, lv)
            if progress:
                progress(e, len(targets) - 1, label)
        b.close()
        for lat in lats:
            lat.close()
        return levels

    fields, flux = {}, {}  # (mesh, base time) -> (rho, T / T_c); -> Q
    Tc0 = [None]
    times = sorted(set(range(0, steps0 + 1, every0)) |
                   set(range(tau0 - m0, tau0 + m0 + 1, shift_every0)))

    def take1(m, e, lat, lv):
        r, _, _, T = lat.fields()
        t = times[e]
        fields[(m, t)] = (r.astype(np.float32), (T / lv["Tc"]).astype(np.float32))
        # lattice units: T scales with T_c(a) ~ dx^2 and d/dy with 1/dx
        if Tc0[0] is None:
            Tc0[0] = lv["Tc"] / (N0 / meshes[0]) ** 2
        flux[(m, t)] = lat.norms()["q_bottom"] * Tc0[0] / (lv["Tc"] * (N0 / meshes[m]))

    levels = march(list(range(nm)), [[int(round(t * q)) for q in ratios] for t in times], take1,
                   "pass 1")
    grid = list(range(0, steps0 + 1, every0))
    out = {"meshes": list(meshes), "steps0": steps0, "every0": every0, "t": grid,
           "kappa": [lv["kappa"] for lv in levels], "sigma": [lv["sigma"] for lv in levels]}
    ratio = meshes[1] / meshes[0]

    def orders(D):
        return [math.log(D[m] / D[m + 1]) / math.log(ratio) for m in range(len(D) - 1)]

    def interp_diff(a, f):
        return float(np.abs(bilinear(a, f.shape) - f).sum())

    for fi, name in ((0, "rho"), (1, "T")):
        out[f"d_{name}"] = [[space_difference(fields[(m, t)][fi], fields[(m + 1, t)][fi]) for t in grid]
                            for m in range(nm - 1)]
        D = [sum(interp_diff(fields[(m, t)][fi], fields[(m + 1, t)][fi]) for t in grid) /
             sum(float(np.abs(fields[(m + 1, t)][fi]).sum()) for t in grid) for m in range(nm - 1)]
        out[f"D_{name}"] = D
        out[f"orders_{name}"] = orders(D)
    # heat flux: t = 0 is left out (a temperature jump at the heater edge,
    # whose one-sided gradient grows as 1 / dx)
    Q = np.array([[flux[(m, t)] for t in grid] for m in range(nm)])
    DQ = [float(np.abs(Q[m, 1:] - Q[m + 1, 1:]).sum() / np.abs(Q[m + 1, 1:]).sum()) for m in range(nm - 1)]
    out["Q"] = Q.tolist()
    out["D_Q"] = DQ
    out["orders_Q"] = orders(DQ)
    out["bubble_area"] = [[float((fields[(m, t)][0][:meshes[m] // 2 - 2] <
                                  0.5 * (levels[m]["rho_l"] + levels[m]["rho_v"])).sum()
                                 * (N0 / meshes[m]) ** 2) for t in grid] for m in range(nm)]
    # Eq. rel-diff-minimize on the density field
    shifts = list(range(-m0, m0 + 1, shift_every0))
    fine = fields[(nm - 1, tau0)][0]
    delta = [best_shift({d: fields[(m, tau0 + d)][0] for d in shifts}, fine, shifts)
             for m in range(nm - 1)] + [0]
    out["delta"] = delta
    # pass 2: shifted samples of every coarser mesh with delta != 0
    shifted = {m: {t: fields[(m, t)] for t in grid} for m in range(nm) if delta[m] == 0}
    redo = [m for m in range(nm) if delta[m] != 0]
    if redo:
        def take2(j, e, lat, lv):
            r, _, _, T = lat.fields()
            shifted.setdefault(redo[j], {})[grid[e]] = (r.astype(np.float32),
                                                        (T / lv["Tc"]).astype(np.float32))
        targets = [[int(round(t * (1 + delta[m] / tau0) * ratios[m])) for m in redo] for t in grid]
        march(redo, targets, take2, "pass 2")
    for fi, name in ((0, "rho"), (1, "T")):
        Ds = [sum(interp_diff(shifted[m][t][fi], shifted[m + 1][t][fi]) for t in grid) /
              sum(float(np.abs(shifted[m + 1][t][fi]).sum()) for t in grid) for m in range(nm - 1)]
        out[f"D_shifted_{name}"] = Ds
        out[f"orders_shifted_{name}"] = orders(Ds)
    return out


def contact_angle(rho, rho_l, rho_v, ymin=3.0, y_wall=0.0):
    """Static contact angle (degrees) of a droplet on the bottom wall: a
    circle fitted by algebraic least squares to the crossings of
    rho = (rho_l + rho_v) / 2 along rows and columns (linear interpolation)
    at heights y >= ymin, and the angle it makes with the wall plane
    y = y_wall inside the liquid, cos(theta) = (y_wall - y_c) / R."""
    import numpy as np

    mid = 0.5 * (rho_l + rho_v)
    ny, nx = rho.shape
    y0 = int(np.ceil(ymin))
    a = rho[y0:] - mid
    pts = []
    # crossings along columns (between rows y and y + 1) and rows
    s = a[:-1] * a[1:] < 0
    yy, xx = np.nonzero(s)
    t = a[yy, xx] / (a[yy, xx] - a[yy + 1, xx])
    pts.append(np.c_[xx, y0 + yy + t])
    s = a[:, :-1] * a[:, 1:] < 0
    yy, xx = np.nonzero(s)
    t = a[yy, xx] / (a[yy, xx] - a[yy, xx + 1])
    pts.append(np.c_[xx + t, y0 + yy])
    P = np.concatenate(pts).astype(float)
    if len(P) < 8:
        raise ValueError("no droplet interface above ymin")
    M = np.c_[2.0 * P, np.ones(len(P))]
    (xc, yc, c), *_ = np.linalg.lstsq(M, (P ** 2).sum(1), rcond=None)
    R = float(np.sqrt(c + xc * xc + yc * yc))
    return float(np.degrees(np.arccos(np.clip((y_wall - yc) / R, -1.0, 1.0))))


def wall_droplet_mesh(N, value, model=0, N0=160, a0=6.12e-2, Tr=0.86, R0_frac=0.25, eta=0.1,
                      precision=0, tile_y=0):
    """Mesh N (N x N) of the contact-angle tests of Sec. 4.3: periodic sides,
    Zou-He walls, isothermal at T_sat = Tr T_c, no gravity; a half disk of
    liquid of radius R0_frac N centred on the bottom wall (smoothed over one
    base-mesh node); bottom wall table = value (rho_w for the psi-based
    model 0, G_w for the modified-psi model 1), top wall rho_w = rho_v or
    G_w = G; a, sigma, kappa by the refinement rules with dx = N0 / N.
    Returns (params, boundary, rho, T, level record)."""
    import numpy as np

    from .sim import make_params, refinement_level

    dx = N0 / N
    lv = refinement_level(a0, dx, Tr, 0.0, 0.0)
    rates = dict(s_rho=1.0, s_e=0.8, s_zeta=0.8, s_j=1.0, s_q=1.1)
    p = make_params(N, N, a=lv["a"], sigma=lv["sigma"], kappa=lv["kappa"], rho_l=lv["rho_l"],
                    rho_v=lv["rho_v"], walls=1, thermal=0, gy=0.0, eta_l=eta, eta_v=eta,
                    rho_ref=lv["rho_v"], wall_model=int(model), precision=precision, tile_y=tile_y,
                    **rates)
    top = lv["rho_v"] if model == 0 else p.G
    bnd = dict(rho_w_bottom=np.full(N, float(value)), rho_w_top=np.full(N, top),
               t_bottom_kind=np.full(N, 1, np.int32), t_bottom_val=lv["T"],
               t_top_kind=np.full(N, 1, np.int32), t_top_val=lv["T"])
    y, x = np.mgrid[0:N, 0:N] + 0.5
    d = np.hypot(x - N / 2, y - 0.5)
    rho = 0.5 * (lv["rho_l"] + lv["rho_v"]) - 0.5 * (lv["rho_l"] - lv["rho_v"]) * np.tanh(
        (d - R0_frac * N) * dx)
    return p, bnd, rho, np.full((N, N), lv["T"]), lv


def wall_droplets(meshes, values, model=0, N0=160, steps0=20000, checks=(0.5, 0.75, 1.0),
                  precision=0, progress=None, keep_fields=False, **kw):
    """Every (mesh, value) droplet of wall_droplet_mesh in one batch, run for
    steps0 base-mesh steps ((N / N0)^2 steps on mesh N).  Returns the
    contact angles at the fractions `checks` of the run (the last one is the
    static angle; the others show whether it has settled) and, with
    keep_fields, the final densities."""
    import numpy as np

    from .sim import Batch, Lattice

    lats, levels, keys = [], [], []
    for N in meshes:
        for v in values:
            p, bnd, rho, T, lv = wall_droplet_mesh(N, v, model, N0, precision=precision, **kw)
            lat = Lattice(p)
            lat.set_boundary(**bnd)
            lat.init_fields(rho, None, None, T)
            lats.append(lat)
            levels.append(lv)
            keys.append((N, v))
    b = Batch(lats)
    angles = np.zeros((len(checks), len(meshes), len(values)))
    fields = {}
    done = [0] * len(lats)
    for k, frac in enumerate(checks):
        target = [int(round(frac * steps0 * (N / N0) ** 2)) for N, _ in keys]
        b.run([t - d for t, d in zip(target, done)])
        done = target
        for j, (lat, lv, (N, v)) in enumerate(zip(lats, levels, keys)):
            r = lat.fields()[0]
            angles[k, j // len(values), j % len(values)] = contact_angle(
                r, lv["rho_l"], lv["rho_v"], ymin=3.0 * N / N0)
            if keep_fields and k == len(checks) - 1:
                fields[(N, v)] = r
        if progress:
            progress(k + 1, len(checks))
    b.close()
    for lat in lats:
        lat.close()
    out = {"meshes": list(meshes), "values": list(values), "model": int(model), "steps0": steps0,
           "checks": list(checks), "angles": angles.tolist()}
    if keep_fields:
        out["fields"] = fields
    return out


def contact_angle_refinement(meshes=(160, 240, 360, 540, 810), rho_w=(4.0, 2.3, 1.7), N0=160,
                             steps0=20000, precision=0, progress=None, **kw):
    """Refinement of the psi-based contact-angle droplets (Sec. 4.3): the
    relative change of the static density fields between consecutive
    meshes, sum |I(rho_N) - rho_N*| / sum |rho_N*| with the bilinear
    interpolation I, its convergence orders, and the static angles."""
    import math

    import numpy as np

    r = wall_droplets(meshes, rho_w, 0, N0, steps0, precision=precision, progress=progress,
                      keep_fields=True, **kw)
    F = r.pop("fields")
    ratio = meshes[1] / meshes[0]
    rel, orders = [], []
    for v in rho_w:
        d = [space_difference(F[(meshes[m], v)], F[(meshes[m + 1], v)]) for m in range(len(meshes) - 1)]
        rel.append(d)
        orders.append([math.log(d[m] / d[m + 1]) / math.log(ratio) for m in range(len(d) - 1)])
    r["rel_change"] = rel
    r["orders"] = orders
    return r


def gw_search(meshes=(160, 240, 360, 540), target=125.9, N0=160, steps0=20000,
              coarse=(-1.0, -0.95, -0.9, -0.85, -0.8, -0.75, -0.7), fine=11, precision=0,
              progress=None, **kw):
    """G_w of the modified-psi model giving the static contact angle
    `target` on each mesh (Sec. 4.3): a linear search over the coarse grid
    (every mesh and value in one batch), then a finer grid of `fine` values
    across the bracketing interval of each mesh, and linear interpolation
    of the angle between the two nearest values."""
    import numpy as np

    coarse = sorted(coarse)
    r1 = wall_droplets(meshes, coarse, 1, N0, steps0, checks=(1.0,), precision=precision,
                       progress=progress, **kw)
    A1 = np.asarray(r1["angles"][0])
    out = {"meshes": list(meshes), "target": target, "coarse": coarse, "coarse_angles": A1.tolist(),
           "gw": [], "fine": [], "fine_angles": []}
    brackets = []
    for m in range(len(meshes)):
        a = A1[m]
        j = next((j for j in range(len(a) - 1) if (a[j] - target) * (a[j + 1] - target) <= 0), None)
        brackets.append(None if j is None else (coarse[j], coarse[j + 1]))
    for m, N in enumerate(meshes):
        if brackets[m] is None:
            out["gw"].append(None)
            out["fine"].append([])
            out["fine_angles"].append([])
            continue
        lo, hi = brackets[m]
        vals = list(np.linspace(lo, hi, fine))
        r2 = wall_droplets((N,), vals, 1, N0, steps0, checks=(1.0,), precision=precision, **kw)
        a = np.asarray(r2["angles"][0][0])
        j = next((j for j in range(len(a) - 1) if (a[j] - target) * (a[j + 1] - target) <= 0), None)
        if j is None:
            gw = None
        else:
            t = (target - a[j]) / (a[j + 1] - a[j]) if a[j + 1] != a[j] else 0.0
            gw = float(vals[j] + t * (vals[j + 1] - vals[j]))
        out["gw"].append(gw)
        out["fine"].append([float(v) for v in vals])
        out["fine_angles"].append(a.tolist())
        if progress:
            progress(m + 1, len(meshes))
    return out


STEFAN_SETS = {
    # Sec. 4.2: first set = the droplet's c_v = 5 with both diffusivities
    # 0.3; second set = c_v = 10, lambda_l = 15, lambda_v = 1
    1: dict(cv=5.0, alpha=0.3),
    2: dict(cv=10.0, lambda_l=15.0, lambda_v=1.0),
}


def stefan_mesh(L, set_id=2, L0=160, a0=6.12e-2, Tr=0.86, Tw_r=0.9, precision=0, tile_y=0):
    """Mesh L of the 1-D boiling problem (Sec. 4.2) as one column of L
    nodes along y: a Zou-He wall at y = 0 held at T_w = Tw_r T_c with the
    psi-based rho_w = rho_v (hydrophobic), a zero-gradient outflow at the
    top (adiabatic temperature), liquid at rest at T_sat = Tr T_c
    everywhere at t = 0; a, sigma, kappa by the refinement rules with
    dx = L0 / L; c_v and the conductivities of parameter set `set_id`.
    Returns (params, boundary, rho, T, level record, thermal constants)."""
    import numpy as np

    from .sim import make_params, refinement_level

    dx = L0 / L
    lv = refinement_level(a0, dx, Tr, 0.0, 0.0)
    st = STEFAN_SETS[set_id]
    cv = st["cv"]
    if "alpha" in st:
        lam_l, lam_v = st["alpha"] * cv * lv["rho_l"], st["alpha"] * cv * lv["rho_v"]
    else:
        lam_l, lam_v = st["lambda_l"], st["lambda_v"]
    rates = dict(s_rho=1.0, s_e=0.8, s_zeta=0.8, s_j=1.0, s_q=1.1)
    p = make_params(1, L, a=lv["a"], sigma=lv["sigma"], kappa=lv["kappa"], rho_l=lv["rho_l"],
                    rho_v=lv["rho_v"], walls=1, outflow_top=1, thermal=1, gy=0.0, cv=cv,
                    lambda_l=lam_l, lambda_v=lam_v, eta_l=0.1, eta_v=0.1, rho_ref=lv["rho_l"],
                    precision=precision, tile_y=tile_y, **rates)
    Tw = Tw_r * lv["Tc"]
    bnd = dict(rho_w_bottom=lv["rho_v"], rho_w_top=lv["rho_v"], t_bottom_kind=np.full(1, 1, np.int32),
               t_bottom_val=Tw, t_top_kind=np.full(1, 2, np.int32), t_top_val=lv["T"])
    rho = np.full((L, 1), lv["rho_l"])
    T = np.full((L, 1), lv["T"])
    th = dict(cv=cv, lambda_l=lam_l, lambda_v=lam_v, Tw=Tw, alpha_v=lam_v / (cv * lv["rho_v"]),
              alpha_l=lam_l / (cv * lv["rho_l"]))
    return p, bnd, rho, T, lv, th


def stefan_front(rho_col, rho_l, rho_v):
    """Interface position (nodes from the wall row): the last crossing of
    (rho_l + rho_v) / 2 from vapour to liquid, linearly interpolated."""
    import numpy as np

    mid = 0.5 * (rho_l + rho_v)
    r = np.asarray(rho_col, dtype=np.float64).ravel()
    k = np.nonzero(r[:-1] < mid)[0]
    if len(k) == 0:
        return 0.0
    k = int(k.max())
    return float(k + (r[k] - mid) / (r[k] - r[k + 1]))


def pr_latent_heat(lv, a, b=2.0 / 21.0, R=1.0, omega=0.344):
    """Latent heat h_fg at the level's T_sat between its Maxwell densities
    (the library's closed form for the EOS)."""
    return _pr_latent_heat(a, lv["T"], lv["rho_v"], lv["rho_l"], b=b, R=R, omega=omega)


def stefan_refinement(meshes=(160, 320, 640, 1280, 2560), sets=(1, 2), L0=160, steps0=40000,
                      every0=200, precision=0, progress=None, **kw):
    """Sec. 4.2 refinement: every (mesh, parameter set) column in one batch,
    the front s(t) in base-mesh nodes sampled every every0 base-mesh steps
    (the same physical times on every mesh), the relative change between
    consecutive meshes sum_t |s_N - s_N*| / sum_t |s_N*| (as for Delta* R in
    Sec. 4.1) with its convergence orders, and the similarity solution
    2 beta sqrt(alpha_v t) (Eq. stefan-analytical) with the Jakob number
    c_v (T_w - T_sat) / h_fg of each set."""
    import math

    import numpy as np

    from .sim import Batch, Lattice

    lats, info = [], []
    for sid in sets:
        for L in meshes:
            p, bnd, rho, T, lv, th = stefan_mesh(L, sid, L0, precision=precision, **kw)
            lat = Lattice(p)
            lat.set_boundary(**bnd)
            lat.init_fields(rho, None, None, T)
            lats.append(lat)
            info.append((sid, L, lv, th, p.a))
    times = list(range(0, steps0 + 1, every0))
    fronts = np.zeros((len(lats), len(times)))
    b = Batch(lats)
    done = [0] * len(lats)
    for k, t in enumerate(times):
        target = [int(round(t * (L / L0) ** 2)) for _, L, _, _, _ in info]
        if k:
            b.run([tg - d for tg, d in zip(target, done)])
        done = target
        for j, (lat, (_, L, lv, _, _)) in enumerate(zip(lats, info)):
            fronts[j, k] = stefan_front(lat.fields()[0][:, 0], lv["rho_l"], lv["rho_v"]) * (L0 / L)
        if progress and k % 20 == 0:
            progress(k, len(times) - 1)
    b.close()
    for lat in lats:
        lat.close()
    out = {"meshes": list(meshes), "t": times, "sets": {}}
    ratio = meshes[1] / meshes[0]
    nm = len(meshes)
    for si, sid in enumerate(sets):
        rows = fronts[si * nm:(si + 1) * nm]
        _, _, lv0, th0, a0_ = info[si * nm]
        hfg = pr_latent_heat(lv0, a0_)
        ja = th0["cv"] * (th0["Tw"] - lv0["T"]) / hfg
        beta = stefan_beta(ja)
        ref = 2.0 * beta * np.sqrt(th0["alpha_v"] * np.asarray(times, dtype=np.float64))
        rel = [float(np.abs(rows[m] - rows[m + 1]).sum() / np.abs(rows[m + 1]).sum())
               for m in range(nm - 1)]
        out["sets"][sid] = {
            "s": rows.tolist(), "reference": ref.tolist(), "ja": ja, "beta": beta,
            "alpha_v": th0["alpha_v"], "alpha_l": th0["alpha_l"],
            "rel_change": rel,
            "orders": [math.log(rel[m] / rel[m + 1]) / math.log(ratio) for m in range(nm - 2)],
            "rel_to_reference": [float(np.abs(r - ref).sum() / np.abs(ref).sum()) for r in rows]}
    return out
