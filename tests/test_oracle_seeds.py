"""Pins of the oracle's SampleSeeds (Algorithm 1; Sec. IV-B: initial
configurations inside the bounds, those that collide at once discarded).

The generator is Philox4x64-10 from its published definition; numpy ships the
same generator (numpy.random.Philox, which advances its 256-bit counter before
each block), so every block is checked against it.  The sampler is then checked
by what the reading fixes: every seed inside the tendon and bending bounds and
zero-sum (extensible robots: the bending part zero-sum and bounded, the length
within its interval), seeds that clear the spheres and the robot itself unless
every attempt collided, attempts counted as documented, a seed that depends only
on (key, problem, seed), and draws that fill the bounds symmetrically."""
import numpy as np
import pytest

from paper_2607_11340_amd import inputs as I


def _numpy_block(ctr, key):
    """The block numpy's Philox returns first for counter ctr - 1 (256-bit)."""
    v = sum(int(c) << (64 * k) for k, c in enumerate(ctr))
    v = (v - 1) % (1 << 256)
    c = np.array([(v >> (64 * k)) & (2 ** 64 - 1) for k in range(4)], dtype=np.uint64)
    return np.random.Philox(counter=c, key=np.array(key, dtype=np.uint64)).random_raw(4)


def test_philox_matches_numpy(oracle):
    rng = np.random.default_rng(1)
    cases = [([0, 0, 0, 0], [0, 0]), ([2 ** 64 - 1, 0, 0, 0], [1, 2]), ([5, 7, 11, 13], [123, 456]),
             ([1, 2 ** 63, 3, 4], [2 ** 64 - 1, 2 ** 64 - 1])]
    cases += [(list(rng.integers(0, 2 ** 63, 4)), list(rng.integers(0, 2 ** 63, 2))) for _ in range(16)]
    for ctr, key in cases:
        assert list(oracle.philox4x64(ctr, key)) == list(_numpy_block(ctr, key)), (ctr, key)


def _robot(oracle, **kw):
    base = dict(L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], u_max=[0.008] * 3, pts_per_seg=8)
    base.update(kw)
    return oracle.Robot(**base)


def _gaps(oracle, ro, u, sph):
    """Smallest sphere clearance and self clearance of configuration u (margin 0)."""
    _, _, pts = oracle.fk(ro, u, points=True)
    p = pts.reshape(-1, 3)
    rad = np.repeat(ro.r, ro.pts_per_seg)
    g = np.inf
    if sph is not None and len(sph):
        g = (np.linalg.norm(p[:, None] - sph[None, :, :3], axis=2) - sph[None, :, 3] - rad[:, None]).min()
    gs = np.inf
    seg = np.repeat(np.arange(ro.n), ro.pts_per_seg)
    far = seg[:, None] >= seg[None, :] + 2
    if far.any():
        d = np.linalg.norm(p[:, None] - p[None], axis=2) - rad[:, None] - rad[None]
        gs = d[far].min()
    return g, gs


def test_seeds_inside_bounds_and_zero_sum(oracle):
    ro = _robot(oracle, theta_max=np.pi)      # the tendon bound binds first
    u, att = oracle.sample_seeds(ro, 5, 400, (7, 9))
    assert (att == 1).all()                                     # nothing to collide with
    assert np.abs(u.sum(axis=3)).max() < 1e-17                  # eq. (4): zero-sum per segment
    assert (np.abs(u) <= np.array(ro.u_max)[:, None] * (1 + 1e-15)).all()
    z = np.array([oracle.u_to_z(ro, x) for x in u.reshape(-1, ro.n, 3)]).reshape(-1, ro.n, 2)
    assert (np.hypot(z[..., 0], z[..., 1]) <= ro.theta_max * (1 + 1e-15)).all()
    # draws fill the bounds and are symmetric: per tendon the largest |u| is close
    # to u_max and the mean is near zero (400 x 5 draws)
    flat = u.reshape(-1, ro.n, 3)
    assert (np.abs(flat).max(axis=0) > 0.95 * np.array(ro.u_max)[:, None]).all()
    assert (np.abs(flat.mean(axis=0)) < 0.1 * np.array(ro.u_max)[:, None]).all()


def test_theta_bound_rejects_and_scales(oracle):
    """A bending bound far below what the tendon bound allows: every seed is cut
    to theta_max, by rejection or, after 32 triples, by scaling."""
    ro = _robot(oracle, theta_max=0.05)
    u, _ = oracle.sample_seeds(ro, 2, 200, (1, 1))
    z = np.array([oracle.u_to_z(ro, x) for x in u.reshape(-1, ro.n, 3)]).reshape(-1, ro.n, 2)
    th = np.hypot(z[..., 0], z[..., 1])
    assert (th <= 0.05 * (1 + 1e-12)).all()
    assert th.max() > 0.045


def test_seed_depends_only_on_key_problem_and_seed(oracle):
    ro = _robot(oracle)
    a, _ = oracle.sample_seeds(ro, 3, 10, (11, 12))
    b, _ = oracle.sample_seeds(ro, 5, 40, (11, 12))
    assert np.array_equal(a, b[:3, :10])
    c, _ = oracle.sample_seeds(ro, 3, 10, (11, 13))
    assert not np.isclose(a, c).any()


def test_colliding_seeds_are_drawn_again(oracle):
    rng = np.random.default_rng(3)
    ro = _robot(oracle)
    # spheres around the workspace of straight-ish configurations
    sph = np.concatenate([rng.uniform([-0.08, -0.08, 0.05], [0.08, 0.08, 0.25], size=(12, 3)),
                          rng.uniform(0.01, 0.03, size=(12, 1))], axis=1)
    P, S, A = 2, 300, 8
    u, att = oracle.sample_seeds(ro, P, S, (5, 6), max_attempts=A, spheres=sph)
    redrawn = 0
    for p in range(P):
        for s in range(S):
            g, _ = _gaps(oracle, ro, u[p, s], sph)
            if att[p, s] > 0:
                assert g >= 0.0, (p, s, att[p, s], g)
            else:
                assert att[p, s] == -A and g < 0.0
            redrawn += abs(att[p, s]) > 1
    assert redrawn > 0                     # the scene makes some first draws collide
    # an attempt that was kept is the one its count names: with max_attempts equal
    # to that count the same seed comes back
    p, s = np.argwhere(att > 1)[0]
    u2, att2 = oracle.sample_seeds(ro, P, S, (5, 6), max_attempts=int(att[p, s]), spheres=sph)
    assert np.array_equal(u2[p, s], u[p, s]) and att2[p, s] == att[p, s]


def test_hopeless_scene_keeps_last_attempt(oracle):
    ro = _robot(oracle)
    sph = np.array([[0.0, 0.0, 0.0, 0.5]])          # engulfs the whole robot
    u, att = oracle.sample_seeds(ro, 1, 20, (2, 2), max_attempts=5, spheres=sph)
    assert (att == -5).all()
    assert (np.abs(u) <= 0.008 * (1 + 1e-15)).all()


def test_extensible_seeds(oracle):
    ro = _robot(oracle, L_min=[0.06, 0.05, 0.04], L_max=[0.12, 0.10, 0.08])
    u, att = oracle.sample_seeds(ro, 2, 300, (4, 4))
    e = u.mean(axis=3)                                     # extension per segment
    bend = u - e[..., None]
    assert (np.abs(bend) <= 0.008 * (1 + 1e-12)).all()
    L = np.array(ro.L) + e
    assert (L >= np.array(ro.L_min) - 1e-15).all() and (L <= np.array(ro.L_max) + 1e-15).all()
    # lengths spread over their whole interval
    span = np.array(ro.L_max) - np.array(ro.L_min)
    assert ((L.reshape(-1, 3).max(axis=0) - L.reshape(-1, 3).min(axis=0)) > 0.9 * span).all()


def test_self_contact_seeds(oracle):
    """A robot whose middle segment may curl back: seeds in self contact are
    drawn again."""
    ro = oracle.Robot(L=[0.08, 0.05, 0.08, 0.06], r=[0.0155, 0.004, 0.0155, 0.006], u_max=[0.01, 0.03, 0.01, 0.01],
                      pts_per_seg=6, theta_max=4.0, self_collision=True)
    u, att = oracle.sample_seeds(ro, 1, 300, (8, 8), max_attempts=8)
    n_redrawn = 0
    for s in range(300):
        _, gs = _gaps(oracle, ro, u[0, s], None)
        assert (gs >= 0.0) == (att[0, s] > 0), (s, gs, att[0, s])
        n_redrawn += abs(att[0, s]) > 1
    assert n_redrawn > 0
