"""One time step of the pseudopotential LBM with phase change, plain and
serial in NumPy float64.

Test infrastructure only (see oracle/__init__.py).

State: populations f[i, y, x] after streaming (pre-collision, the f of
Eq. lbm at t^n) and temperature T[y, x].  Arrays are indexed [y, x]; y = 0
is the bottom row.  x is always periodic; y is periodic or bounded by two
wet-node Zou-He walls at rows 0 and ny-1.

Step n -> n+1 (Sec. 2), in this order:
  1. rho = sum f_i, j = sum f_i c_i                 Eq. DensityAndVelocityRelationToF
  2. rho_bar = mean of rho over all nodes (g != 0)  Eq. gravitational_force
  3. p_EOS, psi at every node; at wall nodes also psi_w = psi(rho_w, T)
                                                    Eqs. peng-robinson, psi, psi-based-formula
  4. F^m = -G psi sum_i W_i psi_nb(i) c_i with psi_nb = psi(x + c_i) for
     fluid neighbours and psi_w(x) for solid ones (this is Eq. shanchen,
     and at wall nodes Eq. shanchen-walls with F^ads of
     Eq. psi-based-formula); F = F^m + g (rho - rho_bar) e_y;
     Q = kappa G/2 psi sum_i W_i (psi_nb(i) - psi) c_i c_i     Eqs. Q, Q-psi-based
     With the modified-psi model the solid neighbours of F^m carry
     (G_w / G) psi(x), which gives F^ads = -G_w psi^2 sum W_i s c_i
     (Eq. mod-psi-based-formula), and those of Q carry psi(x), so that
     they drop out (Eq. Q-mod-psi-based).
  5. u = (j + F/2) / rho                            Eq. DensityAndVelocityRelationToF
  6. m = M f;  m* = m - Lambda (m - m_eq) + (I - Lambda/2) S + C;
     f* = M^-1 m*                                   Eqs. collisionMRT, li_source_terms, S, C
  7. energy equation (if thermal and n >= n_iso), rho and u of step n held:
       T* = T + K(T)/2,  T^{n+1} = T + K(T*)        Eq. energy-equation, RK2
  8. stream f_i(x + c_i) <- f*_i(x); populations that would arrive at a
     wall node from outside the domain are left undefined here and rebuilt
     by the Zou-He closure at the start of the next step (step 1').
  1'. wall nodes (Zou-He, wet node): the known populations give
     K = f0 + f1 + f3 + 2 (f4 + f7 + f8) (bottom; mirror image at the top);
     the closure prescribes the momentum j_w = -F/2 with F = F^m + F^b
     (R4), i.e. zero fluid velocity u = (j + F/2)/rho up to a remainder of
     order |g| |F^m| / ny; its normal component makes the wall density
     solve rho + F_y(rho)/2 = K at the bottom and rho - F_y(rho)/2 = K at
     the top, F_y = F^m_y(rho) + g (rho - rho_bar_K), a scalar equation per
     node (F^m_y depends on the node's own psi and on the adjacent interior
     row only) solved by NEWTON_WALL Newton steps from rho = K; the
     tangential component only splits the unknowns.
     With outflow_top the top row is no wall but a zero-gradient outflow
     (the 1-D boiling problem of Sec. 4.2): after streaming (and at init)
     its populations with c_y < 0 are copied from the row below, psi above
     it is its own (column by column), and it is updated like an interior
     node; its temperature kind is ADIABATIC.

Readings where the paper is silent or garbled (all used identically by
the GPU library):
  R1 the sigma term of S uses |F^m|^2 (the printed "(F^m.F^m)^2" cannot
     be dimensionally right), with F^m the wall-modified interaction force
     (fluid sum + F^ads), never including F^b;
  R2 tau_v in C is the viscous time tau_eta, i.e. C uses s_nu;
  R3 T*_w (wall temperature seen by psi_w) is the node's own T;
  R4 no-slip at a wet node means zero fluid velocity, and the fluid
     velocity of this forcing scheme is u = (sum f c + F/2)/rho
     (Eq. DensityAndVelocityRelationToF), so the Zou-He closure imposes
     sum f c = -F/2 with F = F^m + F^b (F^m including F^ads).  Imposing
     sum f c = 0 instead injects or removes about 3 F_y/4 of mass per wall
     node and step at wetting walls and makes the heated pool unstable.
     The closure's F^b = g (rho - rho_bar_K) takes rho_bar_K, the mean
     density with every wall node counted at its known part K, because the
     closed wall densities cannot enter the buoyancy they balance; the
     wall velocity left is g (rho_bar_K - rho_bar) / (2 rho), of order
     |g| |F^m| / ny (without F^b the closure left F^b/(2 rho), of order
     |g|, and the pool lost mass through both walls);
  R5 rho_bar is the mean of rho^n over every node, before the forces;
  R6 finite differences: grad phi = sum_i W_i phi(x + c_i) c_i and
     lap phi = 6 sum_i w_i (phi(x + c_i) - phi(x)) (isotropic D2Q9), and
     div(lambda grad T) = lambda lap T + grad(lambda) . grad T;
  R7 RK2 is the two-stage midpoint rule; (dp/dT)_rho in stage 2 is taken
     at the stage temperature T*;
  R8 temperature boundary kinds per node: FREE (updated by the scheme),
     DIRICHLET (held at a tabulated value, also applied at init) and
     ADIABATIC (wall-row nodes set to the value of the adjacent interior
     row after every stage); wall rows are never updated by the stencil,
     so no ghost values are needed ("no special treatment", end of Sec. 2.3);
  R9 s_nu follows the viscosity of Eq. eta-rho, s_nu = 1/(3 eta(rho) + 1/2);
  R10 lambda(rho) of Sec. 2.3 uses the coexistence densities rho_l, rho_v
     given in the parameters.

Domain errors (rho <= 0, rho >= 1/b, psi radicand <= 0, T <= 0, NaN) raise
DomainError: the method is undefined there; nothing is clamped.

Parity pins: tests/test_oracle_step.py (conservation invariants, uniform
fixed point, MRT shear-wave viscosity, equal-rate reduction to BGK with
Guo forcing, the energy-moment shifts of the sigma and kappa terms,
buoyancy momentum balance, RK2 Fourier amplification, stencil exactness,
Zou-He momentum, mass conservation (periodic, and at walls under
gravity), planar coexistence vs. Maxwell, the sigma fit and kappa,
Laplace law).
"""
from dataclasses import dataclass, field

import numpy as np

from . import lattice as lat
from .thermo import EOS

FREE, DIRICHLET, ADIABATIC = 0, 1, 2
PSI_BASED, MODIFIED_PSI = 0, 1  # contact-angle models of Sec. 2.2
NEWTON_WALL = 8  # Newton steps of the wall-density equation (fixed count)


class DomainError(ArithmeticError):
    pass


@dataclass
class Params:
    nx: int
    ny: int
    a: float = 2.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    omega: float = 0.344
    G: float = -1.0
    sigma: float = 0.0
    kappa: float = 0.0
    # MRT rates s_rho, s_e, s_zeta, s_j, s_q; s_nu from eta(rho)
    s_rho: float = 1.25
    s_e: float = 1.25
    s_zeta: float = 1.25
    s_j: float = 1.25
    s_q: float = 1.25
    eta_l: float = 0.1
    eta_v: float = 0.1
    rho_l: float = 6.5  # coexistence densities for eta(rho), lambda(rho)
    rho_v: float = 0.38
    gy: float = 0.0  # gravity along y (negative = downwards)
    walls: bool = False  # Zou-He walls at y = 0 and y = ny-1
    # contact-angle model of the walls (Sec. 2.2): PSI_BASED uses the wall
    # densities rho_w (Eq. psi-based-formula), MODIFIED_PSI the adhesion
    # strengths G_w (Eq. mod-psi-based-formula); per column
    wall_model: int = 0
    rho_w_bottom: np.ndarray = None  # [nx] psi-based wall densities
    rho_w_top: np.ndarray = None
    gw_bottom: np.ndarray = None  # [nx] modified-psi adhesion strengths
    gw_top: np.ndarray = None
    # the top row is a zero-gradient outflow (Sec. 4.2, after Lou et al.)
    # instead of a Zou-He wall: its populations entering from above are
    # those of the row below, and psi above it is its own
    outflow_top: bool = False
    thermal: bool = False
    n_iso: int = 0  # first n_iso steps keep T frozen
    cv: float = 5.0
    lambda_l: float = 2.0 / 3.0
    lambda_v: float = 2.0 / 3.0
    # temperature boundary description
    t_bottom_kind: np.ndarray = None  # [nx] FREE/DIRICHLET/ADIABATIC for row 0
    t_bottom_val: np.ndarray = None
    t_top_kind: np.ndarray = None  # [nx] for row ny-1
    t_top_val: np.ndarray = None
    t_side_dirichlet: bool = False  # columns 0 and nx-1 held at t_side_val
    t_side_val: float = 0.0

    def __post_init__(self):
        nx = self.nx
        def col(v, fill, dt=np.float64):
            if v is None:
                return np.full(nx, fill, dtype=dt)
            if dt is np.float64 and np.iscomplexobj(v):
                dt = np.complex128  # complex-step differentiation (oracle/adjoint.py)
            v = np.asarray(v, dtype=dt)
            return np.full(nx, v, dtype=dt) if v.ndim == 0 else v.copy()
        self.rho_w_bottom = col(self.rho_w_bottom, 1.0)
        self.rho_w_top = col(self.rho_w_top, 1.0)
        self.gw_bottom = col(self.gw_bottom, self.G)
        self.gw_top = col(self.gw_top, self.G)
        if self.wall_model not in (PSI_BASED, MODIFIED_PSI):
            raise ValueError("wall_model must be PSI_BASED or MODIFIED_PSI")
        if self.outflow_top and not self.walls:
            raise ValueError("outflow_top needs walls (a Zou-He wall at the bottom)")
        self.t_bottom_kind = col(self.t_bottom_kind, FREE, np.int64)
        self.t_top_kind = col(self.t_top_kind, FREE, np.int64)
        self.t_bottom_val = col(self.t_bottom_val, 0.0)
        self.t_top_val = col(self.t_top_val, 0.0)

    @property
    def eos(self):
        return EOS(self.a, self.b, self.R, self.omega, self.G)


class Sim:
    """Oracle simulation: init_fields / step / fields / populations / norms."""

    def __init__(self, params: Params, dtype=np.float64):
        self.p = params
        self.eos = params.eos
        self.dtype = dtype
        ny, nx = params.ny, params.nx
        self.f = np.zeros((9, ny, nx), dtype=dtype)
        self.T = np.zeros((ny, nx), dtype=dtype)
        self.n = 0
        self._build_tkind()

    # ------------------------------------------------------------------ setup
    def _build_tkind(self):
        p = self.p
        ny, nx = p.ny, p.nx
        kind = np.zeros((ny, nx), dtype=np.int64)
        val = np.zeros((ny, nx), dtype=np.result_type(p.t_bottom_val, p.t_top_val, np.float64))
        kind[0, :] = p.t_bottom_kind
        val[0, :] = p.t_bottom_val
        kind[ny - 1, :] = p.t_top_kind
        val[ny - 1, :] = p.t_top_val
        if p.t_side_dirichlet:
            for x in (0, nx - 1):
                kind[:, x] = DIRICHLET
                val[:, x] = p.t_side_val
        self.tkind, self.tval = kind, val

    def apply_t_bc(self, T):
        """Rule R8 on a new temperature (or RK stage) field, in place."""
        ny = self.p.ny
        d = self.tkind == DIRICHLET
        T[d] = self.tval[d]
        ab = self.tkind[0, :] == ADIABATIC
        if ab.any():  # (a lattice of one row has no row above its bottom row)
            T[0, ab] = T[1, ab]
        at = self.tkind[ny - 1, :] == ADIABATIC
        if at.any():
            T[ny - 1, at] = T[ny - 2, at]
        return T

    def init_fields(self, rho, ux=None, uy=None, T=None):
        """f := f_eq(rho, u) (Eq. EquilibriumDistribution); T given, then the
        Dirichlet values of R8 are applied."""
        rho = np.asarray(rho, dtype=self.dtype)
        ux = np.zeros_like(rho) if ux is None else np.asarray(ux, dtype=self.dtype)
        uy = np.zeros_like(rho) if uy is None else np.asarray(uy, dtype=self.dtype)
        self.f = self.apply_outflow(feq_weights(rho, ux, uy))
        Tin = np.asarray(T, dtype=self.dtype).copy()
        if self.p.thermal:  # R8: Dirichlet values hold from the start
            d = self.tkind == DIRICHLET
            Tin[d] = self.tval[d]
        self.T = Tin
        self.n = 0

    # ----------------------------------------------------------------- pieces
    def moments(self, f):
        rho = f.sum(axis=0)
        jx = np.tensordot(lat.CX.astype(float), f, axes=(0, 0))
        jy = np.tensordot(lat.CY.astype(float), f, axes=(0, 0))
        return rho, jx, jy

    def check_domain(self, rho, T, rad):
        bad = ~(rho > 0) | ~(rho < 1.0 / self.p.b) | ~(T > 0) | ~(rad > 0)
        if np.any(bad):
            raise DomainError("state leaves the domain of the EOS / pseudopotential "
                              f"at {int(np.count_nonzero(bad))} nodes (step {self.n})")

    def psi_fields(self, rho, T):
        """psi at every node and psi_w at every node of a wall row."""
        rad = self.eos.psi_radicand(rho, T)
        self.check_domain(np.real(rho), np.real(T), np.real(rad))
        psi = np.sqrt(rad)
        psi_w_bot = psi_w_top = None
        if self.p.walls:
            ny = self.p.ny
            psi_w_bot = self.eos.psi(self.p.rho_w_bottom, T[0, :])
            psi_w_top = self.eos.psi(self.p.rho_w_top, T[ny - 1, :])
        return psi, psi_w_bot, psi_w_top

    def neighbour_psi(self, psi, psi_w_bot, psi_w_top):
        """psi_nb[i][y, x] = psi(x + c_i), or the given solid value at x
        (one per column and wall) if x + c_i is solid."""
        ny = self.p.ny
        nb = []
        for i in range(9):
            v = np.roll(psi, (-lat.CY[i], -lat.CX[i]), axis=(0, 1)).copy()
            if self.p.walls:
                if lat.CY[i] < 0:
                    v[0, :] = psi_w_bot
                if lat.CY[i] > 0:
                    if self.p.outflow_top:  # zero gradient: the row above is the top row
                        v[ny - 1, :] = np.roll(psi[ny - 1], -lat.CX[i])
                    else:
                        v[ny - 1, :] = psi_w_top
            nb.append(v)
        return nb

    def forces(self, rho, psi, nb, nbq, rho_bar):
        """nb: neighbour psi seen by F^m (solid neighbours carry psi_w, or
        (G_w / G) psi(x) for the modified model, which turns G psi psi_nb
        into the G_w psi^2 of Eq. mod-psi-based-formula); nbq: neighbour psi
        seen by Q (Eq. Q-psi-based, or psi(x) itself for solid neighbours
        under Eq. Q-mod-psi-based)."""
        G = self.p.G
        sx = sum(lat.W_INT[i] * nb[i] * lat.CX[i] for i in range(1, 9))
        sy = sum(lat.W_INT[i] * nb[i] * lat.CY[i] for i in range(1, 9))
        fmx = -G * psi * sx
        fmy = -G * psi * sy
        fx = fmx
        fy = fmy + self.p.gy * (rho - rho_bar)
        k = self.p.kappa * G / 2.0 * psi
        d = [nbq[i] - psi for i in range(9)]
        qxx = k * sum(lat.W_INT[i] * d[i] * lat.CX[i] * lat.CX[i] for i in range(1, 9))
        qyy = k * sum(lat.W_INT[i] * d[i] * lat.CY[i] * lat.CY[i] for i in range(1, 9))
        qxy = k * sum(lat.W_INT[i] * d[i] * lat.CX[i] * lat.CY[i] for i in range(1, 9))
        return fmx, fmy, fx, fy, qxx, qyy, qxy

    def s_nu(self, rho):
        p = self.p
        eta = ((rho - p.rho_v) * p.eta_l + (p.rho_l - rho) * p.eta_v) / (p.rho_l - p.rho_v)
        return 1.0 / (3.0 * eta + 0.5)

    def collide(self, f, rho, ux, uy, fx, fy, fmx, fmy, psi, qxx, qyy, qxy):
        """Eqs. collisionMRT + li_source_terms: returns f*."""
        p = self.p
        snu = self.s_nu(rho)
        m = np.tensordot(lat.M, f, axes=(1, 0))
        meq = meq_moments(rho, ux, uy)
        tau_e, tau_z = 1.0 / p.s_e, 1.0 / p.s_zeta
        fm2 = fmx * fmx + fmy * fmy
        uf = ux * fx + uy * fy
        S = np.stack([
            np.zeros_like(rho),
            6.0 * uf + 12.0 * p.sigma * fm2 / (psi * psi * (tau_e - 0.5)),
            -6.0 * uf - 12.0 * p.sigma * fm2 / (psi * psi * (tau_z - 0.5)),
            fx, -fx, fy, -fy,
            2.0 * (ux * fx - uy * fy),
            ux * fy + uy * fx,
        ])
        zero = np.zeros_like(rho)
        C = np.stack([
            zero,
            1.5 * p.s_e * (qxx + qyy),
            -1.5 * p.s_zeta * (qxx + qyy),
            zero, zero, zero, zero,
            -snu * (qxx - qyy),
            -snu * qxy,
        ])
        lam = [np.full_like(rho, v) for v in
               (p.s_rho, p.s_e, p.s_zeta, p.s_j, p.s_q, p.s_j, p.s_q)] + [snu, snu]
        lam = np.stack(lam)
        mstar = m - lam * (m - meq) + (1.0 - lam / 2.0) * S + C
        return np.tensordot(lat.M_INV, mstar, axes=(1, 0))

    # ------------------------------------------------------- energy equation
    @staticmethod
    def grad(phi):
        gx = sum(lat.W_INT[i] * np.roll(phi, (-lat.CY[i], -lat.CX[i]), axis=(0, 1)) * lat.CX[i]
                 for i in range(1, 9))
        gy = sum(lat.W_INT[i] * np.roll(phi, (-lat.CY[i], -lat.CX[i]), axis=(0, 1)) * lat.CY[i]
                 for i in range(1, 9))
        return gx, gy

    @staticmethod
    def lap(phi):
        return 6.0 * sum(lat.W_EQ[i] * (np.roll(phi, (-lat.CY[i], -lat.CX[i]), axis=(0, 1)) - phi)
                         for i in range(1, 9))

    def conductivity(self, rho):
        p = self.p
        return (p.lambda_l * (rho - p.rho_v) + p.lambda_v * (p.rho_l - rho)) / (p.rho_l - p.rho_v)

    def energy_rhs(self, Tf, rho, ux, uy):
        """K(T) of Eq. energy-equation with rho, u held (R6, R7)."""
        p = self.p
        gTx, gTy = self.grad(Tf)
        lapT = self.lap(Tf)
        lam = self.conductivity(rho)
        glx, gly = self.grad(lam)
        dux, _ = self.grad(ux)
        _, duy = self.grad(uy)
        divu = dux + duy
        rcv = rho * p.cv
        return (-(ux * gTx + uy * gTy) + (lam * lapT + glx * gTx + gly * gTy) / rcv
                - Tf * self.eos.dp_dT(rho, Tf) * divu / rcv)

    def energy_update(self, T, rho, ux, uy):
        Ts = self.apply_t_bc(T + 0.5 * self.energy_rhs(T, rho, ux, uy))
        return self.apply_t_bc(T + self.energy_rhs(Ts, rho, ux, uy))

    # -------------------------------------------------------------- streaming
    def stream(self, fstar):
        f = np.empty_like(fstar)
        for i in range(9):
            f[i] = np.roll(fstar[i], (lat.CY[i], lat.CX[i]), axis=(0, 1))
        return self.apply_outflow(f)

    def apply_outflow(self, f):
        """Zero-gradient outflow of the top row: the populations that would
        enter it from above are those of the row below (in place)."""
        if self.p.outflow_top:
            ny = self.p.ny
            for i in range(9):
                if lat.CY[i] < 0:
                    f[i, ny - 1] = f[i, ny - 2]
        return f

    # ------------------------------------------------------------- full step
    def known_parts(self, f):
        """Known part K of the density of each wall row (bottom, top; None
        for an outflow top): K = f0 + f1 + f3 + 2 (f4 + f7 + f8) at the
        bottom, its mirror image at the top."""
        ny = self.p.ny
        b = f[:, 0, :]
        kb = b[0] + b[1] + b[3] + 2.0 * (b[4] + b[7] + b[8])
        if self.p.outflow_top:
            return kb, None
        t = f[:, ny - 1, :]
        return kb, t[0] + t[1] + t[3] + 2.0 * (t[2] + t[5] + t[6])

    def mean_known_density(self, f):
        """rho_bar_K of the closure (R4): the mean density with each wall
        node counted at its known part K (the closure's own result cannot
        enter the buoyancy it balances)."""
        ny = self.p.ny
        kb, kt = self.known_parts(f)
        top = f[:, ny - 1, :].sum(axis=0) if kt is None else kt
        tot = kb.sum() + f[:, 1:ny - 1, :].sum() + top.sum()
        return tot / (self.p.nx * ny)

    def wall_closure(self, f, T, rho_bar_k=0.0):
        """Step 1': returns (rho_bottom, rho_top) of the two wall rows; the
        unknown populations are rebuilt later by close_populations once F^m
        at the wall nodes is known.  The prescribed momentum is -F/2 with
        F = F^m + F^b, F^b = g (rho - rho_bar_k) (R4)."""
        p, eos, G, ny = self.p, self.eos, self.p.G, self.p.ny
        gy = p.gy
        rho_int = f[:, 1:ny - 1, :].sum(axis=0)
        psi_int = eos.psi(rho_int, T[1:ny - 1, :])
        out = []
        rows = [(0, 1, +1, p.rho_w_bottom), (ny - 1, ny - 2, -1, p.rho_w_top)]
        if p.outflow_top:
            rows = rows[:1]
            out = [None]  # no closure at the top: its density is the plain sum
        kb, kt = self.known_parts(f)
        for row, adj, sgn, rw in rows:
            K = kb if sgn > 0 else kt
            pa = psi_int[adj - 1]
            # F^m_y: fluid neighbours in the adjacent row (weights 1/3,
            # 1/12, 1/12, c_y = sgn), solid ones (c_y = -sgn, weights summing
            # to 1/2)
            nbsum = pa / 3.0 + (np.roll(pa, -1) + np.roll(pa, 1)) / 12.0
            r = K.copy()
            # the normal component: bottom rho + F_y / 2 = K, top
            # rho - F_y / 2 = K, with F_y = F^m_y(rho) + g (rho - rho_bar_k)
            if p.wall_model == PSI_BASED:
                # F^m_y = psi(rho) B with psi_w for the solid neighbours
                pw = eos.psi(rw, T[row])
                B = -G * sgn * (nbsum - 0.5 * pw)
                for _ in range(NEWTON_WALL):
                    g = r + sgn * 0.5 * (eos.psi(r, T[row]) * B + gy * (r - rho_bar_k)) - K
                    dg = 1.0 + sgn * 0.5 * (eos.dpsi_drho(r, T[row]) * B + gy)
                    r = r - g / dg
            else:
                # Eq. mod-psi-based-formula: F^m_y = sgn (-G psi nbsum +
                # G_w psi^2 / 2)
                gw = p.gw_bottom if sgn > 0 else p.gw_top
                for _ in range(NEWTON_WALL):
                    ps = eos.psi(r, T[row])
                    dps = eos.dpsi_drho(r, T[row])
                    g = (r + 0.5 * (-G * ps * nbsum + 0.5 * gw * ps * ps)
                         + sgn * 0.5 * gy * (r - rho_bar_k) - K)
                    dg = 1.0 + 0.5 * (-G * nbsum + gw * ps) * dps + sgn * 0.5 * gy
                    r = r - g / dg
            out.append(r)
        return (out[1], out[0]) if p.outflow_top else (out[0], out[1])

    @staticmethod
    def close_populations(f, jxw_b, jyw_b, jxw_t, jyw_t):
        """Zou-He reconstruction of the unknown populations of the two wall
        rows for prescribed momenta (jxw, jyw); in place on f."""
        ny = f.shape[1]
        b = f[:, 0, :]
        d = 0.5 * (b[1] - b[3])
        b[2] = b[4] + (2.0 / 3.0) * jyw_b
        b[5] = b[7] - d + 0.5 * jxw_b + jyw_b / 6.0
        b[6] = b[8] + d - 0.5 * jxw_b + jyw_b / 6.0
        t = f[:, ny - 1, :]
        d = 0.5 * (t[1] - t[3])
        t[4] = t[2] - (2.0 / 3.0) * jyw_t
        t[7] = t[5] + d - 0.5 * jxw_t - jyw_t / 6.0
        t[8] = t[6] - d + 0.5 * jxw_t - jyw_t / 6.0

    def macro(self, f=None, T=None):
        """Steps 1'-5: returns a dict of the fields at t^n (and the closed
        populations under key 'f')."""
        f = self.f if f is None else f
        T = self.T if T is None else T
        p = self.p
        f = f.copy()
        rho, jx, jy = self.moments(f)
        rho_bar_k = 0.0
        if p.walls:
            if p.gy != 0.0:
                rho_bar_k = self.mean_known_density(f)
            rb, rt = self.wall_closure(f, T, rho_bar_k)
            rho[0, :] = rb
            if not p.outflow_top:
                rho[p.ny - 1, :] = rt
        rho_bar = rho.mean() if p.gy != 0.0 else 0.0
        psi, pwb, pwt = self.psi_fields(rho, T)
        if p.walls and p.wall_model == MODIFIED_PSI:
            ny = p.ny
            nb = self.neighbour_psi(psi, p.gw_bottom / p.G * psi[0], p.gw_top / p.G * psi[ny - 1])
            nbq = self.neighbour_psi(psi, psi[0], psi[ny - 1])
        else:
            nb = nbq = self.neighbour_psi(psi, pwb, pwt)
        fmx, fmy, fx, fy, qxx, qyy, qxy = self.forces(rho, psi, nb, nbq, rho_bar)
        if p.walls:
            ny = p.ny
            top = f[:, ny - 1].copy()
            # prescribed wall momentum -(F^m + F^b)/2, F^b with rho_bar_k (R4)
            fby = [p.gy * (rho[row] - rho_bar_k) for row in (0, ny - 1)]
            self.close_populations(f, -0.5 * fmx[0], -0.5 * (fmy[0] + fby[0]),
                                   -0.5 * fmx[ny - 1], -0.5 * (fmy[ny - 1] + fby[1]))
            for row, fb in (((0, fby[0]),) if p.outflow_top else ((0, fby[0]), (ny - 1, fby[1]))):
                jx[row] = -0.5 * fmx[row]
                jy[row] = -0.5 * (fmy[row] + fb)
            if p.outflow_top:
                f[:, ny - 1] = top
        ux = (jx + 0.5 * fx) / rho
        uy = (jy + 0.5 * fy) / rho
        return dict(f=f, rho=rho, jx=jx, jy=jy, rho_bar=rho_bar, psi=psi, fmx=fmx, fmy=fmy,
                    fx=fx, fy=fy, qxx=qxx, qyy=qyy, qxy=qxy, ux=ux, uy=uy)

    def step(self, nsteps=1):
        for _ in range(nsteps):
            m = self.macro()
            fstar = self.collide(m["f"], m["rho"], m["ux"], m["uy"], m["fx"], m["fy"],
                                 m["fmx"], m["fmy"], m["psi"], m["qxx"], m["qyy"], m["qxy"])
            if self.p.thermal and self.n >= self.p.n_iso:
                self.T = self.energy_update(self.T, m["rho"], m["ux"], m["uy"])
            self.f = self.stream(fstar)
            self.n += 1
        return self

    # ------------------------------------------------------------ read-back
    def fields(self):
        m = self.macro()
        return m["rho"], m["ux"], m["uy"], self.T.copy()

    def populations(self):
        """Populations at t^n after the wall closure."""
        return self.macro()["f"]

    def norms(self):
        """Global diagnostics of the state at t^n.

        mass, mean, L1 (mean |.|), L2 (rms) and Linf (max |.|) of rho and T,
        max |u|, and two bottom-wall heat fluxes built on lambda dT/dy at
        y = 0 with the one-sided second-order difference
        (-3 T_0 + 4 T_1 - T_2) / 2 (Eq. pool-heat-flux, sign as printed):
          q_bottom -- (1/nx) times its sum over the bottom nodes; an
                      adiabatic node has no flux by its condition and adds 0
          q_heater -- its mean over the held (Dirichlet) bottom nodes: the
                      heater of a heated strip in an adiabatic wall, the
                      quantity a heater Nusselt number is built on
        Nodes whose rho, u or T is not finite are counted and left out."""
        m = self.macro()
        rho, ux, uy = np.real(m["rho"]), np.real(m["ux"]), np.real(m["uy"])
        T = np.real(self.T)
        n = rho.size
        fin = np.isfinite(rho) & np.isfinite(T) & np.isfinite(ux) & np.isfinite(uy)
        r, t = rho[fin], T[fin]
        umag = np.sqrt(ux[fin] ** 2 + uy[fin] ** 2)
        out = dict(mass=float(r.sum()), rho_mean=float(r.sum() / n),
                   umax=float(umag.max()) if umag.size else 0.0,
                   l1_rho=float(np.abs(r).sum() / n), l2_rho=float(np.sqrt((r * r).sum() / n)),
                   linf_rho=float(np.abs(r).max()) if r.size else 0.0,
                   l1_T=float(np.abs(t).sum() / n), l2_T=float(np.sqrt((t * t).sum() / n)),
                   linf_T=float(np.abs(t).max()) if t.size else 0.0,
                   nonfinite=int(n - np.count_nonzero(fin)), q_bottom=0.0, q_heater=0.0,
                   n_heater=0, step=self.n)
        if self.p.walls:
            kind = self.tkind[0]
            lam = self.conductivity(rho[0])
            flux = lam * (-3.0 * T[0] + 4.0 * T[1] - T[2]) / 2.0
            ok = fin[0] & (kind != ADIABATIC)
            held = fin[0] & (kind == DIRICHLET)
            out["q_bottom"] = float(flux[ok].sum() / self.p.nx)
            out["n_heater"] = int(np.count_nonzero(held))
            out["q_heater"] = float(flux[held].mean()) if held.any() else 0.0
        return out


# ---------------------------------------------------------------- helpers
def meq_moments(rho, ux, uy):
    """M f_eq: the equilibrium moments (projection of
    Eq. EquilibriumDistribution on the rows of M)."""
    u2 = ux * ux + uy * uy
    return np.stack([
        rho,
        rho * (-2.0 + 3.0 * u2),
        rho * (1.0 - 3.0 * u2),
        rho * ux, -rho * ux,
        rho * uy, -rho * uy,
        rho * (ux * ux - uy * uy),
        rho * ux * uy,
    ])


def feq_weights(rho, ux, uy):
    """Eq. EquilibriumDistribution in its weight form, c_s^2 = 1/3."""
    out = []
    u2 = ux * ux + uy * uy
    for i in range(9):
        cu = lat.CX[i] * ux + lat.CY[i] * uy
        out.append(lat.W_EQ[i] * (rho + 3.0 * rho * cu + 4.5 * rho * cu * cu - 1.5 * rho * u2))
    return np.stack(out)
