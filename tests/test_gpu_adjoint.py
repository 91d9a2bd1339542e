"""The library's hand-written adjoint (heater-profile gradient of the
evaporated liquid mass) against the oracle's complex-step gradient, central
differences of the library's own float64 forward, and torch.autograd."""
import numpy as np
import pytest

import cases
from oracle import adjoint as oadj

pytestmark = pytest.mark.gpu


def _problem(c, rho, T, nsteps, ckpt, precision=0, rho_ref=None):
    from paper_2201_04560_amd import HeaterProblem

    p = cases.lib_params(c, precision=precision, rho_ref=rho_ref)
    bnd = dict(t_bottom_kind=c["t_bottom_kind"].astype(np.int32), t_bottom_val=c["t_bottom_val"],
               t_top_kind=c["t_top_kind"].astype(np.int32), t_top_val=c["t_top_val"])
    return HeaterProblem(p, bnd, rho, T, nsteps, ckpt)


def _oracle_grad(c, rho, T, n, rm, w, entries=None):
    g = oadj.heater_gradient(cases.oracle_params(c), rho, T, n, rm, w, entries)
    return g


@pytest.mark.parametrize("nsteps,ckpt", [(12, 5), (12, 12), (12, 1)])
def test_adjoint_fp64_matches_oracle_gradient(nsteps, ckpt):
    """16 x 14, all 16 heater entries, ragged last segment / one segment /
    a checkpoint every step."""
    print(f"case adjoint tiny nsteps={nsteps} ckpt={ckpt}", flush=True)
    c, rho, T, rm, w = cases.heater_case()
    pr = _problem(c, rho, T, nsteps, ckpt)
    J = pr.run(c["t_bottom_val"])
    g = pr.adjoint.backward(1.0)
    Jo = oadj.evaporated_mass(cases.oracle_params(c), rho, T, nsteps, rm, w)
    go = _oracle_grad(c, rho, T, nsteps, rm, w)
    go = np.array([go[x] for x in range(c["nx"])])
    errJ = abs(J - Jo) / abs(Jo)
    errg = np.abs(g - go).max() / np.abs(go).max()
    print(f"J {J:.12e} oracle {Jo:.12e} rel {errJ:.2e}; grad rel {errg:.2e}", flush=True)
    assert errJ < 1e-12
    assert errg < 1e-10
    assert g[0] == 0.0 and g[-1] == 0.0


@pytest.mark.parametrize("precision", [0, 1])
def test_adjoint_with_isothermal_start(precision):
    """16 x 14, energy equation off for the first 5 of 12 steps (segments of
    5, 5, 2): the reversed steps before n_iso have no energy adjoint and their
    recompute no first RK stage.  Float64 storage against the oracle's
    complex-step gradient; float32 shifted storage against that too: its
    states are rounded to 2^-24 relative each step, 4.4e-7 measured over
    these 12 steps, bound 1e-5."""
    print(f"case adjoint n_iso=5 precision={precision}", flush=True)
    c, rho, T, rm, w = cases.heater_case()
    c = dict(c, n_iso=5)
    pr = _problem(c, rho, T, 12, 5, precision=precision)
    pr.run(c["t_bottom_val"])
    g = pr.adjoint.backward(1.0)
    go = _oracle_grad(c, rho, T, 12, rm, w)
    go = np.array([go[x] for x in range(c["nx"])])
    errg = np.abs(g - go).max() / np.abs(go).max()
    print(f"grad rel {errg:.2e}, max |grad| {np.abs(go).max():.3e}", flush=True)
    assert np.abs(go).max() > 0
    assert errg < (1e-10 if precision == 0 else 1e-5)


def test_adjoint_fp64_medium_against_oracle_entries():
    """56 x 40 (several tiles), 60 steps in segments of 25: four heater
    entries against the oracle's complex-step derivatives."""
    print("case adjoint medium", flush=True)
    c, rho, T, rm, w = cases.heater_case(56, 40, r=9.0, cy=14.0, seed=5)
    pr = _problem(c, rho, T, 60, 25)
    pr.run(c["t_bottom_val"])
    g = pr.adjoint.backward(1.0)
    ent = [5, 20, 28, 41]
    go = _oracle_grad(c, rho, T, 60, rm, w, ent)
    scale = max(abs(v) for v in go.values())
    for x in ent:
        print(x, g[x], go[x], flush=True)
        assert abs(g[x] - go[x]) <= 1e-10 * scale


def test_adjoint_directional_derivative_matches_central_differences():
    """<grad, v> against (J(Tb + h v) - J(Tb - h v)) / 2h of the library's
    float64 forward, h = 1e-4 (a random direction and two unit vectors)."""
    print("case adjoint fd", flush=True)
    c, rho, T, rm, w = cases.heater_case(64, 48, r=10.0, cy=16.0, seed=7)
    pr = _problem(c, rho, T, 100, 50)
    tb = c["t_bottom_val"]
    pr.run(tb)
    g = pr.adjoint.backward(1.0)
    rng = np.random.default_rng(0)
    dirs = [rng.normal(size=c["nx"]), np.eye(c["nx"])[20], np.eye(c["nx"])[33]]
    h = 1e-4
    for v in dirs:
        fd = (pr.run(tb + h * v) - pr.run(tb - h * v)) / (2 * h)
        gv = float(g @ v)
        print(f"fd {fd:.10e} adjoint {gv:.10e}", flush=True)
        assert abs(fd - gv) <= 1e-6 * np.abs(g).sum() + 1e-7 * abs(gv)


def test_adjoint_leaves_forward_end_state_and_repeats():
    print("case adjoint state", flush=True)
    from paper_2201_04560_amd import Lattice

    c, rho, T, rm, w = cases.heater_case(40, 32, r=7.0, cy=12.0, seed=2)
    pr = _problem(c, rho, T, 30, 7)
    pr.run(c["t_bottom_val"])
    end = pr.lattice.populations()
    g1 = pr.adjoint.backward(1.0)
    assert np.array_equal(end, pr.lattice.populations())
    assert pr.lattice.step_count == 30
    g2 = pr.adjoint.backward(-2.5)
    assert np.abs(g2 + 2.5 * g1).max() <= 1e-13 * np.abs(g1).max()
    ref = Lattice(cases.lib_params(c))
    cases.lib_boundary(ref, c)
    ref.init_fields(rho, None, None, T)
    ref.step(30)
    assert np.array_equal(end, ref.populations())


def test_autograd_function():
    print("case adjoint autograd", flush=True)
    import torch

    from paper_2201_04560_amd import evaporated_mass

    c, rho, T, rm, w = cases.heater_case()
    pr = _problem(c, rho, T, 12, 5)
    tb = torch.tensor(c["t_bottom_val"], dtype=torch.float64, requires_grad=True)
    J = evaporated_mass(tb, pr)
    (3.0 * J).backward()
    go = _oracle_grad(c, rho, T, 12, rm, w)
    go = np.array([go[x] for x in range(c["nx"])])
    assert np.abs(tb.grad.numpy() - 3.0 * go).max() <= 1e-10 * np.abs(3.0 * go).max()


@pytest.mark.parametrize("nsteps", [1, 2])
def test_adjoint_dot_product_one_step(nsteps):
    """Adjoint identity of the heater-to-J map over one (and two) steps:
    <grad J, v> from the library's reverse pass equals the oracle's
    complex-step directional derivative dJ/dTb . v (exact to rounding) for
    random directions v, to 1e-12 of |grad J| |v|."""
    print(f"case adjoint dot product nsteps={nsteps}", flush=True)
    c, rho, T, rm, w = cases.heater_case(20, 16, r=4.0, cy=5.0, seed=11)
    pr = _problem(c, rho, T, nsteps, 1)
    pr.run(c["t_bottom_val"])
    g = pr.adjoint.backward(1.0)
    rng = np.random.default_rng(5 + nsteps)
    for _ in range(3):
        v = rng.standard_normal(c["nx"])
        dd = oadj.heater_directional_derivative(cases.oracle_params(c), rho, T, nsteps, rm, w, v)
        print(f"<g, v> {g @ v:.15e} oracle {dd:.15e}", flush=True)
        assert abs(g @ v - dd) <= 1e-12 * np.linalg.norm(g) * np.linalg.norm(v)


def test_adjoint_backward_refuses_a_changed_lattice():
    """A backward after the lattice was stepped, re-initialised or given new
    boundary tables would replay another trajectory: LBM_E_STATE; a new
    forward pass makes it valid again."""
    print("case adjoint stale backward", flush=True)
    from paper_2201_04560_amd import LbmError

    c, rho, T, rm, w = cases.heater_case()
    pr = _problem(c, rho, T, 12, 5)
    pr.run(c["t_bottom_val"])
    g0 = pr.adjoint.backward(1.0)
    pr.lattice.step(1)
    with pytest.raises(LbmError) as ei:
        pr.adjoint.backward(1.0)
    assert ei.value.status == 4
    pr.run(c["t_bottom_val"])
    assert np.array_equal(pr.adjoint.backward(1.0), g0)
    pr.lattice.set_boundary(t_bottom_val=c["t_bottom_val"] * 1.001)
    with pytest.raises(LbmError):
        pr.adjoint.backward(1.0)


def test_autograd_refuses_a_stale_node():
    """Two forward passes of one problem, then the first one's backward:
    its recorded trajectory is gone, so autograd raises instead of returning
    the second trajectory's gradient."""
    print("case adjoint autograd stale", flush=True)
    import torch

    from paper_2201_04560_amd import evaporated_mass

    c, rho, T, rm, w = cases.heater_case()
    pr = _problem(c, rho, T, 12, 5)
    t1 = torch.tensor(c["t_bottom_val"], dtype=torch.float64, requires_grad=True)
    t2 = torch.tensor(c["t_bottom_val"] * 1.002, dtype=torch.float64, requires_grad=True)
    J1 = evaporated_mass(t1, pr)
    J2 = evaporated_mass(t2, pr)
    with pytest.raises(RuntimeError, match="another forward pass"):
        J1.backward()
    J2.backward()
    assert torch.isfinite(t2.grad).all()


def test_adjoint_fp32_storage_tracks_fp64():
    """Float32 shifted storage: the forward and its checkpoints in float32,
    the adjoint arithmetic in float64 at that trajectory (parity unpinned:
    reported and loosely bounded against the float64 gradient)."""
    print("case adjoint fp32", flush=True)
    c, rho, T, rm, w = cases.heater_case(64, 48, r=10.0, cy=16.0, seed=7)
    p64 = _problem(c, rho, T, 100, 50)
    p32 = _problem(c, rho, T, 100, 50, precision=1)
    J64, J32 = p64.run(c["t_bottom_val"]), p32.run(c["t_bottom_val"])
    g64, g32 = p64.adjoint.backward(), p32.adjoint.backward()
    e = np.abs(g32 - g64).max() / np.abs(g64).max()
    print(f"J64 {J64:.8e} J32 {J32:.8e} grad rel {e:.2e}", flush=True)
    assert abs(J32 - J64) <= 1e-4 * abs(J64)
    assert e < 1e-2


def test_adjoint_rejects_unsupported():
    print("case adjoint unsupported", flush=True)
    from paper_2201_04560_amd import HeaterAdjoint, LbmError, Lattice

    c, rho, ux, uy, T = cases.random_tiny(16, 12, seed=1, walls=True, thermal=True)
    lat = Lattice(cases.lib_params(c))
    with pytest.raises(LbmError) as ei:
        HeaterAdjoint(lat, 10, 5)
    assert ei.value.status == 6


@pytest.mark.slow
def test_adjoint_full_size_entry_vs_oracle():
    """The measured configuration (256^2 droplet vaporisation, 500 steps,
    checkpoint every 50) in float64 storage: the centre heater entry against
    one complex-step run of the oracle (about half a minute on the host)."""
    print("case adjoint 256^2 x 500, entry 128", flush=True)
    import workloads as wl

    eos, Tsat, rv, rl = cases.coexistence()
    Tout = 0.95 * eos.Tc
    n = 256
    c = dict(nx=n, ny=n, a=2.0 / 49.0, sigma=0.1, kappa=0.1, rho_l=rl, rho_v=rv, thermal=True,
             cv=6.0, lambda_l=2 / 3, lambda_v=2 / 3, t_side_dirichlet=True, t_side_val=Tout,
             t_bottom_kind=np.full(n, 1), t_bottom_val=np.full(n, Tout),
             t_top_kind=np.full(n, 1), t_top_val=np.full(n, Tout), **cases.wl.DROPLET_RATES)
    rho, T = wl.droplet(n, n, 30.0, 4.6 / 5.0, rl, rv, Tsat, Tout, seed=0)
    rm, w = 0.5 * (rl + rv), (rl - rv) / 8.0
    pr = _problem(c, rho, T, 500, 50)
    pr.run(c["t_bottom_val"])
    g = pr.adjoint.backward()
    go = _oracle_grad(c, rho, T, 500, rm, w, [128])[128]
    print(f"entry 128: adjoint {g[128]:.12e} oracle {go:.12e}", flush=True)
    assert abs(g[128] - go) <= 1e-9 * np.abs(g).max()
