"""Reverse mode of the time step behind torch.autograd: the gradient of the
evaporated liquid mass with respect to the heater profile (the bottom-row
Dirichlet temperatures), computed by the library's hand-written adjoint
kernels with step checkpointing.  PyTorch supplies the device buffers and
the autograd plumbing only."""
import ctypes

import numpy as np

from . import _native as nat
from ._native import check, lib
from .sim import Lattice


class HeaterAdjoint:
    """Forward / backward passes over nsteps steps of one lattice.

    J = M_l(start) - M_l(end), M_l = sum rho H(rho), H the smooth liquid
    indicator (1 + tanh((rho - rho_mid) / width)) / 2; defaults: rho_mid
    halfway between the coexistence densities, width an eighth of their gap."""

    def __init__(self, lattice, nsteps, ckpt_every=50, rho_mid=None, width=None):
        import torch

        p = lattice.p
        self.lattice = lattice
        self.nsteps, self.ckpt_every = int(nsteps), int(ckpt_every)
        self.rho_mid = 0.5 * (p.rho_l + p.rho_v) if rho_mid is None else float(rho_mid)
        self.width = (p.rho_l - p.rho_v) / 8.0 if width is None else float(width)
        n = ctypes.c_size_t()
        check(lib().lbm_adjoint_bytes(ctypes.byref(p), self.nsteps, self.ckpt_every, ctypes.byref(n)),
              None, "lbm_adjoint_bytes")
        self._buf = torch.empty(n.value + 256, dtype=torch.uint8, device=lattice._buf.device)
        aligned = (self._buf.data_ptr() + 255) // 256 * 256
        self.forward_id = 0  # counts forward passes; an autograd node keeps the one it recorded
        self._a = ctypes.c_void_p()
        check(lib().lbm_adjoint_create(lattice._ctx, self.nsteps, self.ckpt_every, self.rho_mid,
                                       self.width, ctypes.c_void_p(aligned), n.value,
                                       ctypes.byref(self._a)), lattice._ctx, "lbm_adjoint_create")

    def forward(self):
        """Advance the lattice by nsteps from its current state; returns J."""
        J = ctypes.c_double()
        self.forward_id += 1
        check(lib().lbm_adjoint_forward(self._a, ctypes.byref(J)), self.lattice._ctx,
              "lbm_adjoint_forward")
        return J.value

    def backward(self, dJ=1.0):
        """dJ * dJ/d t_bottom_val as a float64 array of nx entries."""
        g = np.zeros(self.lattice.nx, dtype=np.float64)
        check(lib().lbm_adjoint_backward(self._a, float(dJ),
                                         g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              self.lattice._ctx, "lbm_adjoint_backward")
        return g

    def timing(self):
        """(forward ms, backward ms) of the last passes, host wall clock."""
        f, b = ctypes.c_double(), ctypes.c_double()
        check(lib().lbm_adjoint_timing(self._a, ctypes.byref(f), ctypes.byref(b)), None,
              "lbm_adjoint_timing")
        return f.value, b.value

    def close(self):
        if getattr(self, "_a", None) is not None and self._a.value:
            lib().lbm_adjoint_destroy(self._a)
            self._a = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HeaterProblem:
    """A fixed lattice set-up (parameters, boundary columns, initial rho and
    T) whose evaporated mass is a function of the heater profile."""

    def __init__(self, params, boundary, rho0, T0, nsteps, ckpt_every=50, rho_mid=None,
                 width=None):
        self.lattice = Lattice(params)
        self.boundary = dict(boundary)
        self.rho0, self.T0 = np.asarray(rho0, np.float64), np.asarray(T0, np.float64)
        self.adjoint = HeaterAdjoint(self.lattice, nsteps, ckpt_every, rho_mid, width)

    def run(self, t_bottom):
        """J for this heater profile (host array of nx values)."""
        bnd = dict(self.boundary)
        bnd["t_bottom_val"] = np.asarray(t_bottom, np.float64)
        self.lattice.set_boundary(**bnd)
        self.lattice.init_fields(self.rho0, None, None, self.T0)
        return self.adjoint.forward()


def _autograd_function():
    import torch

    class EvaporatedMass(torch.autograd.Function):
        """J(t_bottom) with the library's adjoint as its backward."""

        @staticmethod
        def forward(ctx, t_bottom, problem):
            J = problem.run(t_bottom.detach().to("cpu", torch.float64).numpy())
            ctx.problem = problem
            ctx.forward_id = problem.adjoint.forward_id
            ctx.dev, ctx.dtype = t_bottom.device, t_bottom.dtype
            return torch.tensor(J, dtype=torch.float64, device=t_bottom.device)

        @staticmethod
        def backward(ctx, gJ):
            if ctx.problem.adjoint.forward_id != ctx.forward_id:
                raise RuntimeError("evaporated_mass: the problem ran another forward pass after "
                                   "this one; its gradient is gone (backward each result before "
                                   "the next forward, or use one problem per result)")
            g = ctx.problem.adjoint.backward(float(gJ))
            return torch.from_numpy(g).to(ctx.dev, ctx.dtype), None

    return EvaporatedMass


_FN = None


def evaporated_mass(t_bottom, problem):
    """Differentiable evaporated liquid mass of `problem` as a function of
    the heater profile t_bottom (a torch tensor of nx temperatures)."""
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(t_bottom, problem)
