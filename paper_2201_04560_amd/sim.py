"""Python front end of the HIP library: PyTorch provides the device buffer
and the stream, the library does all the work."""
import ctypes

import numpy as np

from . import _native as nat
from ._native import LbmError, LbmNorms, LbmParams, check, lib


def make_params(nx, ny, **kw):
    """LbmParams with the library defaults, overridden by keyword fields."""
    p = LbmParams()
    lib().lbm_default_params(ctypes.byref(p), nx, ny)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def buffer_bytes(p):
    n = ctypes.c_size_t()
    check(lib().lbm_buffer_bytes(ctypes.byref(p), ctypes.byref(n)), None, "lbm_buffer_bytes")
    return n.value


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


class Lattice:
    """One lattice on one GPU (the current torch device)."""

    def __init__(self, params, device=None, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required (torch.cuda.is_available() is False)")
        self.p = params
        self.nx, self.ny = params.nx, params.ny
        dev = torch.device("cuda") if device is None else torch.device(device)
        nbytes = buffer_bytes(params)
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self._buf.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._ctx = ctypes.c_void_p()
        check(lib().lbm_create(ctypes.byref(params), ctypes.c_void_p(aligned), nbytes,
                               ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(self._ctx)),
              None, "lbm_create")

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().lbm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ API
    def set_boundary(self, rho_w_bottom=None, rho_w_top=None, t_bottom_kind=None, t_bottom_val=None,
                     t_top_kind=None, t_top_val=None, gw_bottom=None, gw_top=None):
        """Per-column wall tables: rho_w (psi-based walls) or G_w
        (modified-psi walls, wall_model = 1), and temperature kinds and
        values of the two wall rows; None keeps the current values."""
        nx = self.nx
        if gw_bottom is not None or gw_top is not None:
            if self.p.wall_model != 1:
                raise ValueError("G_w needs wall_model = 1 (modified-psi walls)")
            if rho_w_bottom is not None or rho_w_top is not None:
                raise ValueError("give rho_w or G_w, not both")
            rho_w_bottom, rho_w_top = gw_bottom, gw_top

        def col(v, dt):
            if v is None:
                return None
            v = np.asarray(v, dtype=dt)
            if v.ndim == 0:
                return np.full(nx, v, dtype=dt)
            if v.shape != (nx,):
                raise ValueError(f"boundary column arrays need nx = {nx} entries, got shape {v.shape}")
            return np.ascontiguousarray(v)

        arrs = [col(rho_w_bottom, np.float64), col(rho_w_top, np.float64),
                col(t_bottom_kind, np.int32), col(t_bottom_val, np.float64),
                col(t_top_kind, np.int32), col(t_top_val, np.float64)]
        self._keep = arrs
        ptrs = []
        for a in arrs:
            if a is None:
                ptrs.append(None)
            elif a.dtype == np.int32:
                ptrs.append(a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
            else:
                ptrs.append(_dptr(a))
        check(lib().lbm_set_boundary(self._ctx, *ptrs), self._ctx, "lbm_set_boundary")

    def init_fields(self, rho, ux=None, uy=None, T=None):
        shp = (self.ny, self.nx)
        rho, ux, uy, T = _f64(rho, shp), _f64(ux, shp), _f64(uy, shp), _f64(T, shp)
        check(lib().lbm_init_fields(self._ctx, _dptr(rho), _dptr(ux), _dptr(uy), _dptr(T)),
              self._ctx, "lbm_init_fields")

    def step(self, n=1):
        check(lib().lbm_step(self._ctx, int(n)), self._ctx, "lbm_step")

    def sync(self):
        check(lib().lbm_sync(self._ctx), self._ctx, "lbm_sync")

    def fields(self):
        shp = (self.ny, self.nx)
        out = [np.empty(shp) for _ in range(4)]
        check(lib().lbm_read_fields(self._ctx, *[_dptr(a) for a in out]), self._ctx,
              "lbm_read_fields")
        return tuple(out)

    def populations(self):
        f = np.empty((9, self.ny, self.nx))
        check(lib().lbm_read_populations(self._ctx, _dptr(f)), self._ctx, "lbm_read_populations")
        return f

    def norms(self):
        n = LbmNorms()
        check(lib().lbm_norms(self._ctx, ctypes.byref(n)), self._ctx, "lbm_norms")
        return {k: getattr(n, k) for k, _ in LbmNorms._fields_}

    @property
    def step_count(self):
        return lib().lbm_step_count(self._ctx)

    def last_step_ms(self):
        v = ctypes.c_double()
        check(lib().lbm_last_step_time(self._ctx, ctypes.byref(v)), self._ctx, "lbm_last_step_time")
        return v.value

    def kernel_timing(self, enable=True):
        check(lib().lbm_kernel_timing(self._ctx, int(bool(enable))), self._ctx, "lbm_kernel_timing")

    def kernel_times(self):
        """(sum of step-kernel spans in ms, number of launches) since enabling."""
        s, n = ctypes.c_double(), ctypes.c_int64()
        check(lib().lbm_kernel_times(self._ctx, ctypes.byref(s), ctypes.byref(n)), self._ctx,
              "lbm_kernel_times")
        return s.value, n.value

    @property
    def tile_y(self):
        """Rows per workgroup strip of the step kernel."""
        return lib().lbm_get_tile_y(self._ctx)

    @tile_y.setter
    def tile_y(self, ty):
        check(lib().lbm_set_tile_y(self._ctx, int(ty)), self._ctx, "lbm_set_tile_y")

    @property
    def strip_waves(self):
        """Waves per strip of the energy step (1 or 2; same results)."""
        return lib().lbm_get_strip_waves(self._ctx)

    @strip_waves.setter
    def strip_waves(self, w):
        check(lib().lbm_set_strip_waves(self._ctx, int(w)), self._ctx, "lbm_set_strip_waves")

    def tile_candidates(self, waves=0):
        """Strip heights whose launches fill whole rounds of wave slots on
        this GPU (1..16 waves per SIMD), for `waves` waves per strip (0: the
        current setting).  Ascending."""
        n = ctypes.c_int32()
        check(lib().lbm_tile_candidates(self._ctx, int(waves), None, 0, ctypes.byref(n)), self._ctx,
              "lbm_tile_candidates")
        out = (ctypes.c_int32 * max(n.value, 1))()
        check(lib().lbm_tile_candidates(self._ctx, int(waves), out, n.value, ctypes.byref(n)),
              self._ctx, "lbm_tile_candidates")
        return [int(v) for v in out[:n.value]]

    def autotune_tile_y(self, candidates=(2, 3, 4, 6, 8, 12, 16, 24, 32), steps=20):
        """Time each candidate strip height on this lattice and keep the
        fastest.  The state is saved first and restored afterwards, so the
        simulation is not advanced.  Returns (tile_y, ms per step)."""
        state = self.save_state()
        cand = [int(c) for c in candidates if int(c) >= 2]
        arr = (ctypes.c_int32 * len(cand))(*cand)
        best, ms = ctypes.c_int32(), ctypes.c_double()
        check(lib().lbm_autotune_tile_y(self._ctx, arr, len(cand), int(steps), ctypes.byref(best),
                                        ctypes.byref(ms)), self._ctx, "lbm_autotune_tile_y")
        self.load_state(state)
        self.tile_y = best.value
        return best.value, ms.value

    def save_state(self):
        n = ctypes.c_size_t()
        check(lib().lbm_state_bytes(self._ctx, ctypes.byref(n)), self._ctx, "lbm_state_bytes")
        buf = np.empty(n.value, dtype=np.uint8)
        check(lib().lbm_save_state(self._ctx, buf.ctypes.data_as(ctypes.c_void_p), n.value),
              self._ctx, "lbm_save_state")
        return buf

    def load_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        check(lib().lbm_load_state(self._ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.size),
              self._ctx, "lbm_load_state")


class Batch:
    """Several lattices of one precision and wall setting advanced together:
    each launch steps every lattice that still has steps to do, so the
    coarse meshes of a refinement ladder ride along with the fine ones."""

    def __init__(self, lattices, stream=None):
        import torch

        if not lattices:
            raise ValueError("empty batch")
        self.lattices = list(lattices)
        prec = self.lattices[0].p.precision
        n = ctypes.c_size_t()
        check(lib().lbm_batch_bytes(prec, ctypes.byref(n)), None, "lbm_batch_bytes")
        dev = self.lattices[0]._buf.device
        self._buf = torch.empty(n.value + 256, dtype=torch.uint8, device=dev)
        aligned = (self._buf.data_ptr() + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream(dev)
        ctxs = (ctypes.c_void_p * len(self.lattices))(*[l._ctx.value for l in self.lattices])
        self._b = ctypes.c_void_p()
        st = lib().lbm_batch_create(ctxs, len(self.lattices), ctypes.c_void_p(aligned), n.value,
                                    ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(self._b))
        if st != 0:
            raise LbmError(st, f"lbm_batch_create: {(lib().lbm_last_error(self.lattices[0]._ctx) or b'').decode()}")

    def _check(self, st, what):
        if st != 0:
            detail = lib().lbm_batch_last_error(self._b) or b""
            raise LbmError(st, f"{what}: {detail.decode()}")

    def run(self, steps, use_graph=True):
        """Advance lattice g by steps[g] steps (asynchronous)."""
        if len(steps) != len(self.lattices):
            raise ValueError("one step count per lattice")
        arr = (ctypes.c_int64 * len(steps))(*[int(s) for s in steps])
        self._check(lib().lbm_batch_run(self._b, arr, 1 if use_graph else 0), "lbm_batch_run")

    def prepare(self, steps, use_graph=True):
        """Upload the tables and capture the graphs of run(steps) without
        running it (the following run replays them at once)."""
        if len(steps) != len(self.lattices):
            raise ValueError("one step count per lattice")
        arr = (ctypes.c_int64 * len(steps))(*[int(s) for s in steps])
        self._check(lib().lbm_batch_prepare(self._b, arr, 1 if use_graph else 0), "lbm_batch_prepare")

    def last_time(self):
        """(device ms, step launches, graph launches) of the last run."""
        ms, nl, ng = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().lbm_batch_last_time(self._b, ctypes.byref(ms), ctypes.byref(nl),
                                              ctypes.byref(ng)), "lbm_batch_last_time")
        return ms.value, nl.value, ng.value

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            lib().lbm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ host helpers
def pr_critical_temperature(a, b=2.0 / 21.0, R=1.0):
    return lib().lbm_pr_critical_temperature(a, b, R)


def pr_maxwell(a, T, b=2.0 / 21.0, R=1.0, omega=0.344):
    rv, rl, ps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check(lib().lbm_pr_maxwell(a, b, R, omega, T, ctypes.byref(rv), ctypes.byref(rl),
                               ctypes.byref(ps)), None, "lbm_pr_maxwell")
    return rv.value, rl.value, ps.value


def fit_sigma(a, T, b=2.0 / 21.0, R=1.0, omega=0.344, G=-1.0):
    s = ctypes.c_double()
    check(lib().lbm_fit_sigma(a, b, R, omega, G, T, ctypes.byref(s)), None, "lbm_fit_sigma")
    return s.value


def planar_gamma(a, T, sigma, b=2.0 / 21.0, R=1.0, omega=0.344, G=-1.0):
    g = ctypes.c_double()
    check(lib().lbm_planar_gamma(a, b, R, omega, G, T, sigma, ctypes.byref(g)), None,
          "lbm_planar_gamma")
    return g.value


def pr_latent_heat(a, T, rho_v, rho_l, b=2.0 / 21.0, R=1.0, omega=0.344):
    """Latent heat h_fg at T between the coexistence densities (Sec. 4.2)."""
    h = ctypes.c_double()
    check(lib().lbm_pr_latent_heat(a, b, R, omega, T, rho_v, rho_l, ctypes.byref(h)), None,
          "lbm_pr_latent_heat")
    return h.value


def stefan_beta(ja):
    """beta of Eq. stefan-analytical for the Jakob number ja."""
    v = ctypes.c_double()
    check(lib().lbm_stefan_beta(ja, ctypes.byref(v)), None, "lbm_stefan_beta")
    return v.value


def refinement_level(a_base, dx, Tr=0.86, kappa0=0.0, gy0=0.0, steps0=0, b=2.0 / 21.0, R=1.0,
                     omega=0.344, G=-1.0):
    """Parameters of a mesh dx times the base spacing (Sec. 3): a, T_c, T,
    Maxwell densities, sigma, kappa, target gamma, gravity and step count."""
    L = nat.LbmLevel()
    check(lib().lbm_refinement_level(a_base, dx, Tr, b, R, omega, G, kappa0, gy0, int(steps0),
                                     ctypes.byref(L)), None, "lbm_refinement_level")
    return {k: getattr(L, k) for k, _ in nat.LbmLevel._fields_}
