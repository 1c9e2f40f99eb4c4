"""Pins of the CPU oracle's kinematics against the paper's own formulas written
differently, closed forms and library routines (Sec. III-A eq. 1-3, Sec. III-B eq. 4)."""
import numpy as np
import pytest
from scipy.linalg import expm, logm

from paper_2607_11340_amd import inputs as I

ROB3 = dict(L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], u_max=[0.008] * 3)


def Zrot(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


def Yrot(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, 0, s], [0, 1.0, 0], [-s, 0, c]])


def hom(R, p):
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = R, p
    return T


def tendon_u(theta, phi, r):
    """eq. (4) minus L: u_j = -r theta cos(alpha_j - phi), alpha_j = 2 pi j / 3."""
    al = 2 * np.pi * np.arange(3) / 3
    return -r * theta * np.cos(al - phi)


def test_straight_backbone(oracle):
    rb = oracle.Robot(**ROB3)
    arc, fr = oracle.fk(rb, np.zeros((3, 3)))
    assert np.allclose(fr[-1][:, :3], np.eye(3), atol=0, rtol=0)
    assert np.allclose(fr[-1][:, 3], [0, 0, 0.24], atol=1e-16)
    assert np.all(arc[:, 0] == 0) and np.all(arc[:, 1] == 0)
    # the common mode of a segment's tendons is ignored (inextensible segment)
    arc2, fr2 = oracle.fk(rb, np.full((3, 3), 0.003))
    assert np.abs(fr2 - fr).max() < 1e-15


def test_single_arc_closed_form(oracle):
    """Tip of one arc: ((1-cos kL)/k cos phi, (1-cos kL)/k sin phi, sin(kL)/k)."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        L, r = 0.1, 0.01
        theta, phi = rng.uniform(1e-3, 1.1), rng.uniform(0, 2 * np.pi)
        rb = oracle.Robot(L=[L], r=[r], u_max=[1.0])
        arc, fr = oracle.fk(rb, tendon_u(theta, phi, r)[None])
        k = theta / L
        tip = np.array([(1 - np.cos(k * L)) / k * np.cos(phi), (1 - np.cos(k * L)) / k * np.sin(phi),
                        np.sin(k * L) / k])
        assert np.abs(fr[0][:, 3] - tip).max() < 1e-15
        assert abs(arc[0, 0] - k) < 1e-12 * k and abs(arc[0, 1] - phi) < 1e-12
        # tip tangent (R e_z) is the arc tangent at its end
        tan = np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
        assert np.abs(fr[0][:, 2] - tan).max() < 1e-15


def test_eq2_eq3_literal_and_expm(oracle):
    """Each link T_{i-1}^i equals Z(phi) Y(theta) Z(-phi) with eq. (3)'s d (computed
    from the oracle's own arc parameters), and the exponential of the arc's twist."""
    rb = oracle.Robot(**ROB3)
    rng = np.random.default_rng(4)
    u = I.uniform_actuation(rng, 3, 0.008, 16)
    arc, fr = oracle.fk(rb, u)
    for b in range(16):
        Tprev = np.eye(4)
        for i in range(3):
            kap, phi, L = arc[b, i]
            th = kap * L
            R = Zrot(phi) @ Yrot(th) @ Zrot(-phi)
            d = (L / th) * np.array([np.cos(phi) * (1 - np.cos(th)), np.sin(phi) * (1 - np.cos(th)), np.sin(th)])
            Ti = hom(fr[b, i][:, :3], fr[b, i][:, 3])
            link = np.linalg.solve(Tprev, Ti)
            assert np.abs(link - hom(R, d)).max() < 2e-15
            X = np.zeros((4, 4))
            w = th * np.array([-np.sin(phi), np.cos(phi), 0.0])
            X[:3, :3] = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
            X[2, 3] = L
            assert np.abs(link - expm(X)).max() < 2e-15
            Tprev = Ti


def test_rotations_orthonormal(oracle):
    rb = oracle.Robot(L=[0.08] * 6, r=[0.008] * 6, u_max=[0.01] * 6)
    rng = np.random.default_rng(5)
    u = I.uniform_actuation(rng, 6, 0.01, 32)
    _, fr = oracle.fk(rb, u)
    R = fr[..., :3]
    err = np.abs(np.einsum("...ji,...jk->...ik", R, R) - np.eye(3)).max()
    assert err < 1e-14
    assert np.abs(np.linalg.det(R) - 1).max() < 1e-14


def test_equal_arcs_chain_is_one_arc(oracle):
    """Equal bending plane and equal curvature across segments = one arc of the total length."""
    rng = np.random.default_rng(6)
    for _ in range(10):
        Ls = rng.uniform(0.04, 0.1, size=4)
        kap, phi = rng.uniform(0.5, 4.0), rng.uniform(0, 2 * np.pi)
        rb = oracle.Robot(L=list(Ls), r=[0.01] * 4, u_max=[1.0] * 4)
        u = np.stack([tendon_u(kap * L, phi, 0.01) for L in Ls])
        _, fr = oracle.fk(rb, u)
        Lt = Ls.sum()
        rb1 = oracle.Robot(L=[Lt], r=[0.01], u_max=[1.0])
        _, f1 = oracle.fk(rb1, tendon_u(kap * Lt, phi, 0.01)[None])
        assert np.abs(fr[-1] - f1[0]).max() < 1e-15


def test_tendon_map_round_trip_and_zero_sum(oracle):
    rng = np.random.default_rng(7)
    rb = oracle.Robot(**ROB3)
    for _ in range(50):
        th = rng.uniform(0, 1.2, 3)
        ph = rng.uniform(0, 2 * np.pi, 3)
        u = np.stack([tendon_u(th[i], ph[i], rb.r[i]) for i in range(3)])
        arc, _ = oracle.fk(rb, u + rng.uniform(-0.01, 0.01, size=(3, 1)))  # common mode is irrelevant
        assert np.abs(arc[:, 0] * np.array(rb.L) - th).max() < 1e-13
        dphi = np.angle(np.exp(1j * (arc[:, 1] - ph)))
        assert np.abs(dphi).max() < 1e-12
        z = oracle.u_to_z(rb, u)
        assert np.abs(z - np.stack([th * np.cos(ph), th * np.sin(ph)], 1)).max() < 1e-13
        u2 = oracle.z_to_u(rb, z)
        assert np.abs(u2 - u).max() < 1e-17
        assert np.abs(u2.sum(axis=1)).max() < 1e-17


def test_bending_angle_webster_jones_form(oracle):
    """theta = 2 sqrt(sum u^2 - sum_{j<k} u_j u_k) / (3 r) for three tendons."""
    rng = np.random.default_rng(8)
    rb = oracle.Robot(**ROB3)
    u = rng.uniform(-0.008, 0.008, size=(40, 3, 3))
    arc, _ = oracle.fk(rb, u)
    for b in range(40):
        for i in range(3):
            x = u[b, i]
            q = (x ** 2).sum() - (x[0] * x[1] + x[1] * x[2] + x[0] * x[2])
            th = 2 * np.sqrt(q) / (3 * rb.r[i])
            assert abs(arc[b, i, 0] * rb.L[i] - th) < 1e-13


def test_backbone_points(oracle):
    rng = np.random.default_rng(9)
    rb = oracle.Robot(**ROB3, pts_per_seg=7)
    u = I.uniform_actuation(rng, 3, 0.008, 8)
    arc, fr, pts = oracle.fk(rb, u, points=True)
    assert pts.shape == (8, 3, 7, 3)
    # sigma = 1 point is the segment tip
    assert np.abs(pts[:, :, -1] - fr[:, :, :, 3]).max() < 1e-16
    # points of a segment lie on its circle: distance to the centre of curvature is 1/kappa
    for b in range(8):
        Tprev = np.eye(4)
        for i in range(3):
            kap, phi, _ = arc[b, i]
            c_loc = np.array([np.cos(phi), np.sin(phi), 0.0]) / kap
            c = Tprev[:3, :3] @ c_loc + Tprev[:3, 3]
            d = np.linalg.norm(pts[b, i] - c, axis=1)
            assert np.abs(d - 1 / kap).max() < 1e-14
            Tprev = hom(fr[b, i][:, :3], fr[b, i][:, 3])


def _exp_se3(xi):
    X = np.zeros((4, 4))
    w = xi[3:]
    X[:3, :3] = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    X[:3, 3] = xi[:3]
    return expm(X)


@pytest.mark.parametrize("angle", [1e-9, 1e-5, 0.05, 0.7, 1.3, 2.0, 2.6, 2.9, 3.1, np.pi - 1e-6])
def test_se3_log_residual(oracle, angle):
    """The pose residual is log(T_ee^-1 T_target) (eq. 8/18): with T_target = T_ee exp(xi)
    it must return xi, in every branch of the rotation logarithm."""
    rng = np.random.default_rng(int(angle * 1e6) % 2 ** 31)
    rb = oracle.Robot(**ROB3)
    u = I.uniform_actuation(rng, 3, 0.008, 1)[0]
    z = oracle.u_to_z(rb, u).ravel()
    _, fr = oracle.fk(rb, u)
    Tee = hom(fr[-1][:, :3], fr[-1][:, 3])
    for _ in range(5):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        xi = np.concatenate([rng.normal(size=3) * 0.05, angle * axis])
        Tt = Tee @ _exp_se3(xi)
        W = oracle.Weights(rho_lim=0, rho_curv=0)
        r, _ = oracle.residuals(rb, W, oracle.Problem("ik", Tt[:3]), z)
        assert np.abs(r[:6] - xi).max() < 1e-12 + 1e-9 * (angle > 3.0)
        # independent check with scipy's matrix logarithm
        if angle > 1e-6:
            Lg = np.real(logm(np.linalg.solve(Tee, Tt)))
            ref = np.array([Lg[0, 3], Lg[1, 3], Lg[2, 3], Lg[2, 1], Lg[0, 2], Lg[1, 0]])
            assert np.abs(r[:6] - ref).max() < 1e-8
        e = oracle.pose_error(rb, z.reshape(3, 2), Tt[:3])
        assert abs(e[0] - np.linalg.norm(xi)) < 1e-9
        assert abs(e[1] - np.linalg.norm(Tt[:3, 3] - Tee[:3, 3])) < 1e-15
        assert abs(e[2] - angle) < 1e-9


def test_zero_pose_cost_at_own_fk(oracle):
    rng = np.random.default_rng(10)
    rb = oracle.Robot(**ROB3)
    u = I.uniform_actuation(rng, 3, 0.008, 5)
    _, fr = oracle.fk(rb, u)
    for b in range(5):
        c = oracle.cost(rb, oracle.Weights(), oracle.Problem("ik", fr[b, -1]), u[b])
        assert c < 1e-28
