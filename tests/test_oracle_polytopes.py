"""Pins of the oracle's convex obstacles (the convex pieces of Sec. V's obstacle
model in half-space form; clearance of eq. 10 with the signed distance
sd(x) = max_f (n_f . x - d_f)).

A straight robot (u = 0) has its backbone points on the z axis at heights
k L / K, so the clearance of each point against a box is closed form: against a
face parallel to the axis at distance x0 it is x0 (outside) or minus the depth
(inside); near an edge outside, the reading is the larger of the two face
excesses, which is below the Euclidean distance.  Also: unused planes change
nothing, the collision bit flips where sd - r crosses zero, and central finite
differences of the cost and of the Jacobian with polytope rows active."""
import numpy as np

from paper_2607_11340_amd import inputs as I


def box_planes(c, h, R=np.eye(3), pad=0):
    """Half-spaces of an oriented box (centre c, half extents h, axes the columns
    of R), plus `pad` unused planes (n = 0, d large)."""
    pl = []
    for k in range(3):
        for sgn in (1.0, -1.0):
            n = sgn * R[:, k]
            pl.append(np.concatenate([n, [n @ c + h[k]]]))
    pl += [np.array([0.0, 0.0, 0.0, 1e30])] * pad
    return np.array(pl)


def _straight(oracle, K=8, r=0.005):
    L = [0.10, 0.08]
    rb = oracle.Robot(L=L, r=[r, r], u_max=[0.01, 0.01], pts_per_seg=K)
    z = np.concatenate([np.arange(1, K + 1) / K * L[0], L[0] + np.arange(1, K + 1) / K * L[1]])
    return rb, np.zeros((2, 3)), z


def _penalty(oracle, rb, W, u, poly):
    _, fr = oracle.fk(rb, u)
    T = fr[-1]
    return (oracle.cost(rb, W, oracle.Problem("ik", T, polytopes=poly[None] if poly.ndim == 2 else poly), u)
            - oracle.cost(rb, W, oracle.Problem("ik", T), u))


def test_face_clearance_closed_form(oracle):
    rb, u, zs = _straight(oracle)
    W = oracle.Weights()
    for x0 in (0.0052, 0.0058, 0.0064, 0.010):
        # a slab x >= x0 spanning the robot's height: every point is at sd = x0
        poly = box_planes(np.array([x0 + 0.05, 0.0, 0.1]), np.array([0.05, 0.2, 0.2]))
        viol = W.margin - (x0 - rb.r[0])
        want = 0.5 * W.rho_coll * len(zs) * max(viol, 0.0) ** 2
        got = _penalty(oracle, rb, W, u, poly)
        assert abs(got - want) <= 1e-9 * max(want, 1e-12), (x0, got, want)


def test_inside_clearance_is_minus_depth(oracle):
    """A box that swallows the upper part of the backbone: points inside have
    sd = -(distance to the nearest face)."""
    rb, u, zs = _straight(oracle)
    W = oracle.Weights()
    c, h = np.array([0.003, 0.0, 0.16]), np.array([0.02, 0.03, 0.03])   # z in [0.13, 0.19], x in [-0.017, 0.023]
    poly = box_planes(c, h)
    want = 0.0
    for z in zs:
        p = np.array([0.0, 0.0, z])
        sd = max(np.abs(p - c) - h) if np.all(np.abs(p - c) <= h) else None
        if sd is None:   # outside: the largest face excess
            sd = np.max(np.abs(p - c) - h)
        viol = W.margin - (sd - rb.r[0])
        want += 0.5 * W.rho_coll * max(viol, 0.0) ** 2
    got = _penalty(oracle, rb, W, u, poly)
    assert want > 0 and abs(got - want) <= 1e-9 * want, (got, want)


def test_edge_region_reading(oracle):
    """Outside near an edge the signed distance is the larger face excess (a
    reading of the half-space form), not the Euclidean distance to the edge."""
    rb, u, zs = _straight(oracle, K=4, r=0.004)
    W = oracle.Weights(margin=0.02)
    e = 0.006            # edge parallel to z at (x, y) = (e, e), box in x >= e, y >= e
    poly = box_planes(np.array([e + 0.05, e + 0.05, 0.1]), np.array([0.05, 0.05, 0.2]))
    sd_reading, sd_euclid = e, np.hypot(e, e)
    want = 0.5 * W.rho_coll * len(zs) * (W.margin - (sd_reading - rb.r[0])) ** 2
    got = _penalty(oracle, rb, W, u, poly)
    assert abs(got - want) <= 1e-9 * want
    assert 0.5 * W.rho_coll * len(zs) * (W.margin - (sd_euclid - rb.r[0])) ** 2 < 0.9 * want


def test_unused_planes_and_rotation_change_nothing(oracle):
    rng = np.random.default_rng(5)
    rb = oracle.Robot(L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], u_max=[0.008] * 3, pts_per_seg=6)
    W = oracle.Weights()
    u = I.uniform_actuation(rng, 3, 0.008, 6)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    c, h = np.array([0.02, -0.01, 0.15]), np.array([0.015, 0.02, 0.03])
    a, b = box_planes(c, h, q), box_planes(c, h, q, pad=3)
    # the same box from its 8 vertices' hull written with a plane order reversed
    rev = a[::-1].copy()
    for k in range(6):
        _, fr = oracle.fk(rb, u[k])
        pb = [oracle.Problem("ik", fr[-1], polytopes=x[None]) for x in (a, b, rev)]
        cs = [oracle.cost(rb, W, p_, u[k]) for p_ in pb]
        assert cs[0] == cs[1] and abs(cs[0] - cs[2]) <= 1e-12 * max(cs[0], 1e-12)


def test_collision_bit_flips_at_contact(oracle):
    rb, u, zs = _straight(oracle, K=8, r=0.005)
    _, fr = oracle.fk(rb, u)
    for x0, flagged in ((0.0049, True), (0.0051, False)):
        poly = box_planes(np.array([x0 + 0.05, 0.0, 0.1]), np.array([0.05, 0.2, 0.2]))
        res = oracle.solve(rb, oracle.Weights(), oracle.Problem("ik", fr[-1], polytopes=poly[None]),
                           oracle.Opts(n_final=0, k_init=0, k_final=0), u[None])
        assert bool(res["status"] & oracle.COLLISION) == flagged, (x0, res["status"])


def test_polytope_gradient_and_jacobian_match_fd(oracle):
    rng = np.random.default_rng(9)
    rb = oracle.Robot(L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], u_max=[0.008] * 3, pts_per_seg=6)
    W = oracle.Weights()
    checked = 0
    for k in range(12):
        u = I.uniform_actuation(rng, 3, 0.006, 1)[0]
        _, fr, pts = oracle.fk(rb, u, points=True)
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        # a box whose surface passes near a backbone point of the last segment
        p = pts[2, 3]
        n = q[:, 0]
        h = np.array([0.02, 0.03, 0.03])
        c = p + n * (h[0] + rb.r[2] - 4e-4)
        poly = box_planes(c, h, q)[None]
        _, fr2 = oracle.fk(rb, u + rng.normal(size=(3, 3)) * 2e-4)
        pb = oracle.Problem("ik", fr2[-1], polytopes=poly)
        c0, g = oracle.cost(rb, W, pb, u, grad=True)
        if not c0 > oracle.cost(rb, W, oracle.Problem("ik", fr2[-1]), u) * (1 + 1e-6):
            continue
        checked += 1
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
        assert np.abs(J - Jf).max() <= 1e-5 * np.abs(J).max()
    assert checked >= 6, checked
