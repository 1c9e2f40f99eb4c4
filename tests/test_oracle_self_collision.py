"""Pins of the oracle's self-contact term (eq. 10: the clearance d_min counts
contact between the robot's own segments).  Reading: backbone points of
non-adjacent segments (|i - j| >= 2) keep r_i + r_j apart; the penalty weight and
margin are those of obstacle clearance; the assessment flags CR_COLLISION for a
negative self gap.

A U-shaped robot (segment 0 straight, segment 1 a half circle of radius
rho = L_1 / pi in the x-z plane, segment 2 straight) puts segment 2 parallel to
segment 0 at distance 2 rho, so every pair distance is closed form:
sqrt(4 rho^2 + dz^2).  Also central finite differences of the cost and Jacobian
with the term active, and no change for a robot whose segments stay apart."""
import numpy as np

from paper_2607_11340_amd import inputs as I


def _bend(r, theta, phi=0.0):
    return -r * theta * np.cos(2 * np.pi * np.arange(3) / 3 - phi)


def _u_shape(L, r):
    return np.stack([np.zeros(3), _bend(r[1], np.pi), np.zeros(3)])


def _closed_form_points(L, K):
    """Backbone points of the U shape from geometry alone: segment 0 along +z, the
    half circle ends at (2 rho, 0, L0) heading -z, segment 2 goes down from there."""
    rho = L[1] / np.pi
    s = np.arange(1, K + 1) / K
    p0 = np.stack([np.zeros(K), np.zeros(K), s * L[0]], 1)
    ang = np.pi * s
    p1 = np.stack([rho * (1 - np.cos(ang)), np.zeros(K), L[0] + rho * np.sin(ang)], 1)
    p2 = np.stack([np.full(K, 2 * rho), np.zeros(K), L[0] - s * L[2]], 1)
    return np.stack([p0, p1, p2])


def test_u_shape_points_match_closed_form(oracle):
    L, r, K = [0.08, 0.05, 0.08], [0.008, 0.008, 0.008], 8
    rb = oracle.Robot(L=L, r=r, u_max=[0.1] * 3, pts_per_seg=K, theta_max=4.0)
    _, _, pts = oracle.fk(rb, _u_shape(L, r), points=True)
    assert np.abs(pts - _closed_form_points(L, K)).max() < 1e-15


def test_self_contact_penalty_and_bit_closed_form(oracle):
    L, K, margin, rho_c = [0.08, 0.05, 0.08], 8, 1e-3, 1e6
    d = 2 * L[1] / np.pi                                   # 31.8 mm between segments 0 and 2
    for rr, flagged in ((0.5 * d - 2e-4, False), (0.5 * d + 1e-4, True), (0.5 * d - 4e-4, False)):
        r = [rr, 0.004, rr]
        kw = dict(L=L, r=r, u_max=[0.1] * 3, pts_per_seg=K, theta_max=4.0)
        on, off = oracle.Robot(**kw, self_collision=True), oracle.Robot(**kw)
        u = _u_shape(L, r)
        _, fr = oracle.fk(on, u)
        pb = oracle.Problem("ik", fr[-1])
        W = oracle.Weights(rho_coll=rho_c, margin=margin)
        pts = _closed_form_points(L, K)
        gaps = np.linalg.norm(pts[0][:, None] - pts[2][None], axis=2) - r[0] - r[2]
        want = 0.5 * rho_c * (np.maximum(margin - gaps, 0.0) ** 2).sum()
        got = oracle.cost(on, W, pb, u) - oracle.cost(off, W, pb, u)
        assert abs(got - want) <= 1e-9 * max(want, 1e-12), (rr, got, want)
        assert (want > 0) == (gaps.min() < margin)
        res = oracle.solve(on, W, pb, oracle.Opts(n_final=0, k_init=0, k_final=0), u[None])
        assert bool(res["status"] & oracle.COLLISION) == flagged, (rr, res["status"])
        res = oracle.solve(off, W, pb, oracle.Opts(n_final=0, k_init=0, k_final=0), u[None])
        assert res["status"] == oracle.SOLVED


def test_self_contact_inactive_for_separated_segments(oracle):
    rng = np.random.default_rng(70)
    kw = dict(L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], u_max=[0.008] * 3, pts_per_seg=6)
    on, off = oracle.Robot(**kw, self_collision=True), oracle.Robot(**kw)
    u = I.uniform_actuation(rng, 3, 0.004, 8)
    _, fr = oracle.fk(off, u)
    for k in range(8):
        pb = oracle.Problem("ik", fr[(k + 1) % 8, -1])
        assert oracle.cost(on, oracle.Weights(), pb, u[k]) == oracle.cost(off, oracle.Weights(), pb, u[k])


def test_self_contact_gradient_and_jacobian_match_fd(oracle):
    rng = np.random.default_rng(71)
    L, K = [0.08, 0.05, 0.08, 0.06], 6
    r = [0.0165, 0.004, 0.0165, 0.006]   # 2 L1 / pi = 31.8 mm < r0 + r2: in contact
    rb = oracle.Robot(L=L, r=r, u_max=[0.1] * 4, pts_per_seg=K, theta_max=4.0, self_collision=True)
    W = oracle.Weights()
    base = np.concatenate([_u_shape(L[:3], r[:3]), np.zeros((1, 3))])
    for k in range(4):
        u = base + rng.normal(size=(4, 3)) * 2e-4
        u -= u.mean(axis=1, keepdims=True)
        _, fr = oracle.fk(rb, u + rng.normal(size=(4, 3)) * 3e-4)
        pb = oracle.Problem("ik", fr[-1])
        c, g = oracle.cost(rb, W, pb, u, grad=True)
        off = oracle.Robot(L=L, r=r, u_max=[0.1] * 4, pts_per_seg=K, theta_max=4.0)
        assert c > oracle.cost(off, W, pb, u) * (1 + 1e-6)         # the term is active
        gf = np.zeros_like(u)
        for idx in np.ndindex(u.shape):
            d = np.zeros_like(u)
            d[idx] = 1e-8
            gf[idx] = (oracle.cost(rb, W, pb, u + d) - oracle.cost(rb, W, pb, u - d)) / 2e-8
        assert np.linalg.norm(g - gf) <= 1e-6 * np.linalg.norm(gf), (k, np.linalg.norm(g - gf) / np.linalg.norm(gf))
        z = oracle.u_to_z(rb, u).ravel()
        rv, J = oracle.residuals(rb, W, pb, z)
        Jf = np.zeros_like(J)
        for j in range(z.size):
            d = np.zeros_like(z)
            d[j] = 1e-7
            rp, _ = oracle.residuals(rb, W, pb, z + d)
            rm, _ = oracle.residuals(rb, W, pb, z - d)
            if len(rp) == len(rv) == len(rm):
                Jf[:, j] = (rp - rm) / 2e-7
        assert np.abs(J - Jf).max() <= 1e-6 * np.abs(J).max()
