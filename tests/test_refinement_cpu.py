"""Host-side pieces of the refinement studies (Sec. 4): the coarse-to-fine
interpolation, the relative differences and the time-shift search, against
closed forms; the mesh set-ups against the refinement rules."""
import numpy as np

from paper_2201_04560_amd.ladder import (best_shift, bilinear, droplet_radius, pool_mesh,
                                         space_difference)


def test_bilinear_reproduces_linear_and_constant_fields():
    nc, nf = 16, 24
    yc = (np.arange(nc) + 0.5) / nc
    yf = (np.arange(nf) + 0.5) / nf
    c = np.repeat((3.0 * yc - 1.0)[:, None], nc, axis=1)
    i = bilinear(c, nf)
    exact = np.repeat((3.0 * yf - 1.0)[:, None], nf, axis=1)
    # rows beyond the outermost coarse node centres are clamped
    inner = (yf > yc[0]) & (yf < yc[-1])
    assert np.abs(i - exact)[inner].max() < 1e-14
    assert np.abs(bilinear(np.full((nc, nc), 2.5), nf) - 2.5).max() < 1e-15


def test_bilinear_is_periodic_in_x():
    nc, nf = 12, 18
    xc = 2 * np.pi * (np.arange(nc) + 0.5) / nc
    xf = 2 * np.pi * (np.arange(nf) + 0.5) / nf
    c = np.repeat(np.cos(xc)[None, :], 4, axis=0)
    i = bilinear(c, (6, nf))
    # linear interpolation of cos on a 12-point grid: error below (dx^2 / 8)
    assert np.abs(i - np.cos(xf)[None, :]).max() < (2 * np.pi / nc) ** 2 / 8 + 1e-12


def test_space_difference_and_shift_search():
    n = 32
    y, x = np.mgrid[0:n, 0:n] + 0.5
    front = lambda t: 1.0 + np.tanh((y - 10.0 - 0.01 * t) / 2.0)
    fine = front(600.0)
    assert space_difference(fine, fine) == 0.0
    series = {s: front(600.0 + s) for s in range(-500, 501, 100)}
    assert best_shift(series, fine, list(series)) == 0
    series = {s: front(400.0 + s) for s in range(-500, 501, 100)}
    assert best_shift(series, fine, list(series)) == 200


def test_pool_meshes_follow_the_refinement_rules():
    base = pool_mesh(160)
    for N in (160, 240, 360, 540):
        p, bnd, rho, T, lv = pool_mesh(N)
        dx = 160 / N
        assert abs(p.a / base[0].a - dx ** 2) < 1e-14
        assert abs(p.gy / base[0].gy - dx ** 3) < 1e-14
        hw = int(round(0.05 * N))
        assert (bnd["t_bottom_val"] > lv["T"]).sum() == hw
        assert (bnd["rho_w_bottom"] == 3.44).sum() == hw
        # liquid below half the height, a smooth interface a few base nodes wide
        assert np.abs(rho[:4] - lv["rho_l"]).max() < 1e-9
        assert np.abs(rho[-4:] - lv["rho_v"]).max() < 1e-9
        assert abs(rho[N // 2 - 1, 0] + rho[N // 2, 0] - lv["rho_l"] - lv["rho_v"]) < 1e-12


def test_droplet_radius_of_a_disk():
    n = 200
    y, x = np.mgrid[0:n, 0:n] + 0.5
    d = np.hypot(x - n / 2, y - n / 2)
    rho = 3.44 - 3.06 * np.tanh(d - 40.0)
    assert abs(droplet_radius(rho, 6.5, 0.38) - 40.0) < 0.1


def test_pool_refinement_rejects_fractional_intervals():
    import pytest

    from paper_2201_04560_amd.ladder import pool_refinement

    # 100 base steps are 225 steps on 240 but 506.25 on 360: refused before
    # any lattice is built
    with pytest.raises(ValueError):
        pool_refinement((160, 240, 360), steps0=1000, every0=100, tau0=500, m0=200,
                        shift_every0=100)
    with pytest.raises(ValueError):
        pool_refinement((160, 240), steps0=640, every0=64, tau0=512, m0=256, shift_every0=64)


def test_contact_angle_of_circular_caps():
    """Caps cut from a tanh-profiled disk by the wall plane y = 0 at known
    angles, from hydrophilic to nearly detached."""
    from paper_2201_04560_amd.ladder import contact_angle

    n, R = 220, 40.0
    y, x = np.mgrid[0:n, 0:n] + 0.0
    for th in (30.0, 60.0, 90.0, 125.9, 160.0):
        yc = -R * np.cos(np.radians(th))
        rho = 3.44 - 3.06 * np.tanh(np.hypot(x - 110.0, y - yc) - R)
        assert abs(contact_angle(rho, 6.5, 0.38, ymin=3.0) - th) < 0.2, th


def test_wall_droplet_meshes_follow_the_refinement_rules():
    from paper_2201_04560_amd.ladder import wall_droplet_mesh

    for model, v in ((0, 2.3), (1, -0.9)):
        base = wall_droplet_mesh(160, v, model)
        for N in (160, 240, 360):
            p, bnd, rho, T, lv = wall_droplet_mesh(N, v, model)
            assert p.wall_model == model and p.walls == 1 and p.thermal == 0 and p.gy == 0.0
            assert abs(p.a / base[0].a - (160 / N) ** 2) < 1e-14
            assert np.all(bnd["rho_w_bottom"] == v)
            assert np.all(bnd["rho_w_top"] == (lv["rho_v"] if model == 0 else -1.0))
            # half disk of radius N/4 on the bottom wall
            assert rho[0, N // 2] > lv["rho_l"] - 1e-6 and rho[N // 4 + N // 8, N // 2] < lv["rho_v"] + 1e-3
            assert abs(rho[:, :N // 2].sum() - rho[:, N // 2:][:, ::-1].sum()) < 1e-9 * rho.sum()


def test_stefan_meshes_and_jakob_numbers():
    """Sec. 4.2: both parameter sets give the printed Jakob numbers (0.038,
    0.076) and diffusivities (0.3 / 0.3; 0.23 / 0.26) on every mesh; beta
    solves its transcendental equation."""
    import math

    from paper_2201_04560_amd.ladder import pr_latent_heat, stefan_beta, stefan_front, stefan_mesh

    for sid, ja_p, al, av in ((1, 0.038, 0.3, 0.3), (2, 0.076, 0.23, 0.26)):
        for L in (160, 320, 640):
            p, bnd, rho, T, lv, th = stefan_mesh(L, sid)
            assert p.outflow_top == 1 and p.nx == 1 and p.ny == L and p.gy == 0.0
            ja = th["cv"] * (th["Tw"] - lv["T"]) / pr_latent_heat(lv, p.a)
            assert abs(ja - ja_p) < 1e-3, (sid, L, ja)
            assert abs(th["alpha_l"] - al) < 5e-3 and abs(th["alpha_v"] - av) < 5e-3
            b = stefan_beta(ja)
            assert abs(b * math.exp(b * b) * math.erf(b) * math.sqrt(math.pi) - ja) < 1e-12
    r = np.r_[np.full(7, 0.38), [2.0, 5.0], np.full(20, 6.5)]
    mid = 0.5 * (6.5 + 0.38)
    assert abs(stefan_front(r, 6.5, 0.38) - (7 + (2.0 - mid) / (2.0 - 5.0))) < 1e-12
