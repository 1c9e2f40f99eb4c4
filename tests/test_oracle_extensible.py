"""Pins of the oracle's extensible-segment model (Sec. V-B: extendable robots whose
segment lengths are decision variables within bounds, eq. 9).  Reading: the
common mode of a segment's three tendon displacements is the change of its
length, L_i = L[i] + mean_j u_ij (the mean of eq. 4 over the three tendons is
L_i); the tendon bound applies to the bending part of each displacement and the
length to [L_min, L_max].

* a pure extension (all three tendons equal) gives a straight segment of the new
  length: tip at (0, 0, sum L_i), identity rotation;
* segments of equal curvature and bending plane with different extensions form
  one arc of the total length (closed form of a single arc);
* one extensible segment has a closed-form inverse from its tip position alone
  (theta = 2 atan2(rho, z), phi = atan2(y, x), L = theta |p| / (2 sin(theta/2)));
  the plain solve must recover it;
* the length hinge in closed form, and central finite differences of the cost
  (the common mode now moves the robot) and of every Jacobian column."""
import numpy as np

from paper_2607_11340_amd import inputs as I

ROB = dict(L=[0.08, 0.07, 0.06], r=[0.008, 0.007, 0.006], u_max=[0.006] * 3,
           L_min=[0.06, 0.05, 0.045], L_max=[0.10, 0.09, 0.075])


def _bend(r, theta, phi):
    return -r * theta * np.cos(2 * np.pi * np.arange(3) / 3 - phi)


def _rot_zyz(phi, theta):
    cz, sz, cy, sy = np.cos(phi), np.sin(phi), np.cos(theta), np.sin(theta)
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    return Rz @ Ry @ Rz.T


def test_pure_extension_is_straight(oracle):
    rb = oracle.Robot(**ROB)
    e = np.array([0.013, -0.011, 0.004])
    u = np.repeat(e[:, None], 3, axis=1)
    arc, fr = oracle.fk(rb, u)
    assert np.allclose(arc[:, 2], np.array(ROB["L"]) + e, atol=1e-17, rtol=0)
    assert np.abs(arc[:, 0]).max() < 1e-13   # cos(2 pi j / 3) summed in floating point
    assert np.abs(fr[-1, :, :3] - np.eye(3)).max() < 1e-15
    assert np.abs(fr[-1, :, 3] - [0, 0, sum(ROB["L"]) + e.sum()]).max() < 1e-16
    z = oracle.u_to_z(rb, u)
    assert np.abs(z[:, :2]).max() < 1e-15 and np.allclose(z[:, 2], e, atol=4e-18, rtol=0)
    assert np.abs(oracle.z_to_u(rb, z) - u).max() < 1e-17


def test_equal_curvature_extended_chain_is_one_arc(oracle):
    rb = oracle.Robot(**ROB)
    rng = np.random.default_rng(60)
    for _ in range(5):
        kappa, phi = rng.uniform(0.5, 6.0), rng.uniform(0, 2 * np.pi)
        e = rng.uniform(-0.01, 0.01, size=3)
        Ls = np.array(ROB["L"]) + e
        u = np.stack([_bend(ROB["r"][i], kappa * Ls[i], phi) + e[i] for i in range(3)])
        arc, fr = oracle.fk(rb, u)
        Lt = Ls.sum()
        tip = np.array([(1 - np.cos(kappa * Lt)) / kappa * np.cos(phi), (1 - np.cos(kappa * Lt)) / kappa * np.sin(phi),
                        np.sin(kappa * Lt) / kappa])
        assert np.abs(fr[-1, :, 3] - tip).max() < 1e-15
        assert np.abs(fr[-1, :, :3] - _rot_zyz(phi, kappa * Lt)).max() < 1e-14
        assert np.allclose(arc[:, 0], kappa, rtol=1e-13) and np.allclose(arc[:, 2], Ls, rtol=0, atol=1e-17)


def test_single_extensible_segment_closed_form_ik(oracle):
    """Targets from FK of random (theta, phi, L); 32 uniform seeds, 60 plain
    iterations: the answer equals the closed-form inverse of the tip position."""
    rb = oracle.Robot(L=[0.08], r=[0.008], u_max=[0.008], L_min=[0.05], L_max=[0.11])
    rng = np.random.default_rng(61)
    for _ in range(6):
        th, ph, L = rng.uniform(0.05, 0.9), rng.uniform(0, 2 * np.pi), rng.uniform(0.055, 0.105)
        u_true = (_bend(0.008, th, ph) + (L - 0.08))[None]
        _, fr = oracle.fk(rb, u_true)
        x, y, zz = fr[-1, :, 3]
        th_cf = 2 * np.arctan2(np.hypot(x, y), zz)
        ph_cf = np.arctan2(y, x)
        L_cf = th_cf * np.linalg.norm([x, y, zz]) / (2 * np.sin(th_cf / 2))
        u_cf = _bend(0.008, th_cf, ph_cf) + (L_cf - 0.08)
        assert np.abs(u_cf - u_true[0]).max() < 1e-14
        seeds = I.uniform_actuation(rng, 1, 0.008, 32) + rng.uniform(-0.02, 0.02, size=(32, 1, 1))
        res = oracle.solve(rb, oracle.Weights(), oracle.Problem("ik", fr[-1]),
                           oracle.Opts(n_final=0, k_init=60, k_final=0), seeds)
        assert res["status"] == oracle.SOLVED
        assert np.abs(res["u"][0] - u_cf).max() < 1e-10


def test_length_hinge_closed_form(oracle):
    """A straight configuration extended delta past L_max (other segments inside):
    the length hinge adds rho/2 delta^2; inside the interval it adds nothing."""
    rb = oracle.Robot(**ROB)
    rb_wide = oracle.Robot(**{**ROB, "L_min": [0.0] * 3, "L_max": [1.0] * 3})
    for delta in (3e-4, 2e-3):
        e = np.array([ROB["L_max"][0] - ROB["L"][0] + delta, 0.0, -0.001])
        u = np.repeat(e[:, None], 3, axis=1)
        _, fr = oracle.fk(rb, u)
        pb = oracle.Problem("ik", fr[-1])
        got = oracle.cost(rb, oracle.Weights(), pb, u) - oracle.cost(rb_wide, oracle.Weights(), pb, u)
        assert abs(got - 0.5 * 1e6 * delta ** 2) < 1e-9 * 0.5 * 1e6 * delta ** 2, (delta, got)
    u = np.repeat(np.array([0.001, -0.002, 0.003])[:, None], 3, axis=1)
    _, fr = oracle.fk(rb, u)
    pb = oracle.Problem("ik", fr[-1])
    assert oracle.cost(rb, oracle.Weights(), pb, u) == oracle.cost(rb_wide, oracle.Weights(), pb, u)


def _fd(f, x, h):
    g = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        d = np.zeros_like(x)
        d[idx] = h
        g[idx] = (f(x + d) - f(x - d)) / (2 * h)
    return g


def test_extensible_gradient_and_jacobian_match_fd(oracle):
    rng = np.random.default_rng(62)
    rb = oracle.Robot(**{**ROB, "u_max": [0.003] * 3, "theta_max": 0.5,
                         "L_max": [0.085, 0.075, 0.064]})   # bending, tendon and length hinges active
    W = oracle.Weights()
    targets = I.uniform_actuation(rng, 3, 0.006, 3)
    _, fr = oracle.fk(oracle.Robot(**ROB), targets)
    sph = np.array([[0.02, 0.01, 0.12, 0.02], [-0.03, 0.0, 0.18, 0.015]])
    for k in range(3):
        u = I.uniform_actuation(rng, 3, 0.006, 1)[0] + rng.uniform(0.0, 0.008, size=(3, 1))
        for pb in (oracle.Problem("ik", fr[k, -1]), oracle.Problem("ik", fr[k, -1], spheres=sph)):
            c, g = oracle.cost(rb, W, pb, u, grad=True)
            gf = _fd(lambda x: oracle.cost(rb, W, pb, x), u, 1e-8)
            assert np.linalg.norm(g - gf) <= 1e-6 * np.linalg.norm(gf), (k, g, gf)
            assert np.abs(g.sum(axis=1)).max() > 1e-6 * np.abs(g).max()  # the common mode counts now
            z = oracle.u_to_z(rb, u).ravel()
            r, J = oracle.residuals(rb, W, pb, z)
            Jf = np.zeros_like(J)
            for j in range(z.size):
                d = np.zeros_like(z)
                d[j] = 1e-7
                rp, _ = oracle.residuals(rb, W, pb, z + d)
                rm, _ = oracle.residuals(rb, W, pb, z - d)
                if len(rp) == len(r) == len(rm):
                    Jf[:, j] = (rp - rm) / 2e-7
            assert np.abs(J - Jf).max() <= 1e-6 * np.abs(J).max()
            # J^T r is the gradient in z: through z(u) it equals dC/du
            gz = (J.T @ r).reshape(3, 3)
            Ainv = np.stack([-np.cos(2 * np.pi * np.arange(3) / 3), -np.sin(2 * np.pi * np.arange(3) / 3)])
            gu = np.stack([gz[i, :2] @ (Ainv / (1.5 * rb.r[i])) + gz[i, 2] / 3.0 for i in range(3)])
            assert np.abs(gu - g).max() <= 1e-9 * np.abs(g).max()
