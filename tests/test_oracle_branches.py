"""Pins of the CPU oracle's remaining branches, each against something other than
the oracle itself:

* Levenberg-Marquardt (Sec. IV-C): the backtracking branch (full step rejected by
  the Armijo test, half step taken, damping kept) and the all-rejected branch
  (iterate kept, damping times ten), with the step from numpy.linalg.lstsq of the
  damped stacked system and the Armijo test evaluated on the residual vector;
* the tendon velocity / acceleration hinges of eq. (13)-(14) in closed form on
  actuations linear and quadratic in time;
* the assessment bits of the success test (Sec. V-B with 1 mm / 1 degree): limit
  and bending bounds just inside / outside, a straight backbone beside a sphere
  (closed-form gap), target offsets just inside / outside the thresholds;
* the exploration stage of path following (Sec. IV-B): on a single-segment robot
  every assembled waypoint equals the closed-form inverse of its reference pose,
  and a hand-built case fixes the assembly rule (nearest successful candidate in
  the infinity norm, ties to the lower seed, nearest finite fallback, previous
  waypoint when nothing is finite)."""
import numpy as np

from paper_2607_11340_amd import inputs as I

ROB3 = dict(L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], u_max=[0.008] * 3)
ARMIJO = 1e-4


def _damped_step(oracle, rb, W, pb, z0, lam):
    r, J = oracle.residuals(rb, W, pb, z0)
    D = np.maximum(np.diag(J.T @ J), 1e-12)
    A = np.vstack([J, np.diag(np.sqrt(lam * D))])
    d = np.linalg.lstsq(A, np.concatenate([-r, np.zeros(z0.size)]), rcond=None)[0]
    return d, 0.5 * r @ r, J.T @ r


def _half_cost(oracle, rb, W, pb, z):
    r, _ = oracle.residuals(rb, W, pb, z)
    return 0.5 * r @ r


def _ik_draws(oracle, seed, count):
    rng = np.random.default_rng(seed)
    rb = oracle.Robot(**ROB3)
    for _ in range(count):
        u = I.uniform_actuation(rng, 3, 0.008, 2)
        _, fr = oracle.fk(rb, u)
        yield rb, oracle.Problem("ik", fr[0, -1]), oracle.u_to_z(rb, u[1]).ravel()


def test_lm_backtracking_takes_half_step(oracle):
    """A case whose full damped step fails the Armijo test and whose half step
    passes: the oracle moves by exactly delta / 2 and keeps lambda."""
    W, lam = oracle.Weights(), 1e-6
    hits = 0
    for rb, pb, z0 in _ik_draws(oracle, 5, 60):
        z1, lam1, _, failed, trials = oracle.lm(rb, W, pb, oracle.Opts(), z0, lam, 1)
        if trials != 2:
            continue
        d, c0, g = _damped_step(oracle, rb, W, pb, z0, lam)
        gd = g @ d
        assert _half_cost(oracle, rb, W, pb, z0 + d) > c0 + ARMIJO * gd
        assert _half_cost(oracle, rb, W, pb, z0 + 0.5 * d) <= c0 + ARMIJO * 0.5 * gd
        assert not failed and lam1 == lam
        assert np.abs((z1 - z0) - 0.5 * d).max() <= 1e-9 * np.abs(d).max()
        hits += 1
    assert hits >= 2, hits


def test_lm_all_trials_rejected_keeps_iterate(oracle):
    """A case where every trial step 1, 1/2, 1/4, 1/8 fails the Armijo test: z is
    unchanged and lambda grows tenfold."""
    W, lam = oracle.Weights(), 1e-6
    hits = []
    for rb, pb, z0 in _ik_draws(oracle, 5, 60):
        z1, lam1, _, failed, trials = oracle.lm(rb, W, pb, oracle.Opts(), z0, lam, 1)
        if trials != 4 or not np.array_equal(z1, z0):
            continue
        d, c0, g = _damped_step(oracle, rb, W, pb, z0, lam)
        gd = g @ d
        for a in (1.0, 0.5, 0.25, 0.125):
            assert _half_cost(oracle, rb, W, pb, z0 + a * d) > c0 + ARMIJO * a * gd, a
        assert not failed and lam1 == 10 * lam
        hits.append((rb, pb, z0))
    assert len(hits) >= 1, len(hits)
    # the same rejected step with lambda already at its ceiling: lambda stays there
    rb, pb, z0 = hits[0]
    z2, lam2, _, _, _ = oracle.lm(rb, W, pb, oracle.Opts(lambda_max=lam), z0, lam, 1)
    assert lam2 == lam and np.array_equal(z2, z0)


def _zero_sum(rng, n):
    x = rng.uniform(-1.0, 1.0, size=(n, 3))
    return x - x.mean(axis=1, keepdims=True)


def test_velocity_hinge_closed_form_linear_actuation(oracle):
    """u_t = u_0 + t v: every tendon velocity is v / dt and every acceleration 0, so
    switching on v_max adds sum_t sum_m rho/2 max(0, |v_m|/dt - v_max)^2 and a_max
    adds nothing."""
    rng = np.random.default_rng(41)
    n, H, dt, rho = 2, 5, 0.7, 1e6
    rb = oracle.Robot(L=[0.08] * n, r=[0.008] * n, u_max=[0.006] * n)
    u0 = 1e-3 * _zero_sum(rng, n)
    v = 4e-4 * _zero_sum(rng, n)
    u = np.stack([u0 + t * v for t in range(H + 1)])
    _, fr = oracle.fk(rb, u)
    pb = oracle.Problem("path", fr[:, -1], H=H)
    base = dict(dt=dt, rho_lim=rho)
    c_off = oracle.cost(rb, oracle.Weights(**base), pb, u)
    vel = np.abs(v).ravel() / dt
    for vmax in (0.5 * vel.max(), 0.9 * vel.min(), 2 * vel.max()):
        want = H * 0.5 * rho * (np.maximum(vel - vmax, 0.0) ** 2).sum()
        got = oracle.cost(rb, oracle.Weights(v_max=vmax, **base), pb, u) - c_off
        assert abs(got - want) <= 1e-9 * max(want, c_off), (vmax, got, want)
    got = oracle.cost(rb, oracle.Weights(a_max=1e-9, **base), pb, u) - c_off
    assert abs(got) <= 1e-12 * c_off


def test_acceleration_hinge_closed_form_quadratic_actuation(oracle):
    """u_t = u_0 + t^2 c: velocity (2t - 1) c / dt at t >= 1, acceleration 2 c / dt^2
    at t >= 2; each hinge's share of the cost in closed form."""
    rng = np.random.default_rng(42)
    n, H, dt, rho = 3, 6, 1.3, 2e5
    rb = oracle.Robot(L=[0.08] * n, r=[0.008] * n, u_max=[0.006] * n)
    u0 = 5e-4 * _zero_sum(rng, n)
    cq = 4e-5 * _zero_sum(rng, n)
    u = np.stack([u0 + t * t * cq for t in range(H + 1)])
    _, fr = oracle.fk(rb, u)
    pb = oracle.Problem("path", fr[:, -1], H=H)
    base = dict(dt=dt, rho_lim=rho)
    c_off = oracle.cost(rb, oracle.Weights(**base), pb, u)
    acc = 2 * np.abs(cq).ravel() / dt ** 2
    amax = 0.6 * acc.max()
    want = (H - 1) * 0.5 * rho * (np.maximum(acc - amax, 0.0) ** 2).sum()
    got = oracle.cost(rb, oracle.Weights(a_max=amax, **base), pb, u) - c_off
    assert want > 0 and abs(got - want) <= 1e-9 * max(want, c_off), (got, want)
    vel = np.abs(cq).ravel()[None, :] * (2 * np.arange(1, H + 1) - 1)[:, None] / dt
    vmax = 0.5 * vel.max()
    want = 0.5 * rho * (np.maximum(vel - vmax, 0.0) ** 2).sum()
    got = oracle.cost(rb, oracle.Weights(v_max=vmax, **base), pb, u) - c_off
    assert want > 0 and abs(got - want) <= 1e-9 * max(want, c_off), (got, want)


def _assess(oracle, rb, pb, u):
    """Status of one configuration: a plain solve of zero iterations from it."""
    res = oracle.solve(rb, oracle.Weights(), pb, oracle.Opts(n_final=0, k_init=0, k_final=0), np.asarray(u)[None])
    return res["status"], res["err"]


def _bend(r, theta, phi=0.0):
    """Zero-sum tendon displacements of one segment bent by theta in plane phi
    (eq. 4: u_j = -r theta cos(alpha_j - phi))."""
    return -r * theta * np.cos(2 * np.pi * np.arange(3) / 3 - phi)


def test_assessment_limit_bits(oracle):
    b, r = 0.008, 0.010
    for excess, flagged in ((2e-6, True), (0.5e-6, False)):
        th = (b + excess) / r       # the tendon at alpha = 0 reaches b + excess
        u = _bend(r, th)[None]
        rb = oracle.Robot(L=[0.1], r=[r], u_max=[b])
        _, fr = oracle.fk(rb, u)
        st, err = _assess(oracle, rb, oracle.Problem("ik", fr[-1]), u)
        assert bool(st & oracle.LIMIT_VIOLATION) == flagged, (excess, st)
        assert st == (oracle.LIMIT_VIOLATION if flagged else oracle.SOLVED)
        assert err[0] < 1e-15 and err[1] < 1e-7
    th = 0.5
    u = _bend(r, th, 1.0)[None]
    for tmax, flagged in ((th - 1e-9, True), (th + 1e-9, False)):
        rb = oracle.Robot(L=[0.1], r=[r], u_max=[b], theta_max=tmax)
        _, fr = oracle.fk(rb, u)
        st, _ = _assess(oracle, rb, oracle.Problem("ik", fr[-1]), u)
        assert bool(st & oracle.LIMIT_VIOLATION) == flagged, (tmax, st)


def test_assessment_collision_bit_straight_backbone(oracle):
    """Straight backbone: points (0, 0, k L / K).  A sphere of radius R centred at
    (x0, 0, 0.05) is nearest to the point at z = 0.05, so the clearance is
    x0 - R - r exactly; the check uses margin 0 (the cost's 1 mm margin does not
    count)."""
    L, r, R, K = 0.1, 0.01, 0.02, 10
    rb = oracle.Robot(L=[L], r=[r], u_max=[0.01], pts_per_seg=K)
    u = np.zeros((1, 3))
    _, fr = oracle.fk(rb, u)
    for gap, flagged in ((-1e-5, True), (1e-5, False), (5e-4, False)):
        sph = np.array([[R + r + gap, 0.0, 0.05, R]])
        pb = oracle.Problem("ik", fr[-1], spheres=sph)
        st, _ = _assess(oracle, rb, pb, u)
        assert st == (oracle.COLLISION if flagged else oracle.SOLVED), (gap, st)
        # the cost sees the 1 mm margin: its clearance share is rho/2 (margin - gap)^2
        c_with = oracle.cost(rb, oracle.Weights(), pb, u)
        want = 0.5 * 1e6 * (1e-3 - gap) ** 2
        assert abs(c_with - want) <= 1e-9 * want, (gap, c_with, want)


def test_assessment_convergence_thresholds(oracle):
    """Targets offset from the reached pose by 0.5 / 1.5 mm and 0.8 / 1.2 degrees."""
    rng = np.random.default_rng(43)
    rb = oracle.Robot(**ROB3)
    u = I.uniform_actuation(rng, 3, 0.008, 1)[0]
    _, fr = oracle.fk(rb, u)
    T = fr[-1]
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    for off, flagged in ((0.5e-3, False), (1.5e-3, True)):
        Tq = T.copy()
        Tq[:, 3] += off * d
        st, err = _assess(oracle, rb, oracle.Problem("ik", Tq), u)
        assert bool(st & oracle.NOT_CONVERGED) == flagged and abs(err[0] - off) < 1e-15, (off, st, err)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    for deg, flagged in ((0.8, False), (1.2, True)):
        a = np.radians(deg)
        Rq = np.eye(3) + np.sin(a) * Kx + (1 - np.cos(a)) * Kx @ Kx
        Tq = T.copy()
        Tq[:, :3] = T[:, :3] @ Rq
        st, err = _assess(oracle, rb, oracle.Problem("ik", Tq), u)
        assert bool(st & oracle.NOT_CONVERGED) == flagged and abs(err[1] - a) < 1e-12, (deg, st, err)
        assert err[0] < 1e-15


def _single_arc_z(T):
    """Closed-form inverse of one arc leaving the origin along +z."""
    x, y, zz = T[:, 3]
    th = 2 * np.arctan2(np.hypot(x, y), zz)
    ph = np.arctan2(y, x)
    return np.array([th * np.cos(ph), th * np.sin(ph)])


def test_path_seeds_single_segment_closed_form(oracle):
    """n = 1: the IK solution of every waypoint is unique, so every assembled path
    equals the closed-form inverse of the reference poses, whatever the seeds."""
    rng = np.random.default_rng(44)
    rb = oracle.Robot(L=[0.10], r=[0.010], u_max=[0.010])
    H, S = 5, 4
    uref = I.smooth_actuation_paths(rng, 1, 0.010, 1, H + 1)[0]
    _, fr = oracle.fk(rb, uref)
    seeds = I.uniform_actuation(rng, 1, 0.010, S * (H + 1)).reshape(S, H + 1, 1, 3)
    z = oracle.path_seeds(rb, oracle.Weights(), oracle.Problem("path", fr[:, -1], H=H), oracle.Opts(), seeds, 100)
    want = np.stack([_single_arc_z(fr[t, -1]) for t in range(H + 1)])
    assert np.abs(z[:, :, 0, :] - want[None]).max() <= 1e-9


def test_path_seeds_assembly_rule_hand_case(oracle):
    """Zero IK iterations, so each candidate is its seed.  Single segment, five
    waypoints, three seeds; d = 2e-3 rad moves the tip by about 0.1 mm (a success),
    0.15 rad and more fail.  Hand-worked sources (seed index) per path and waypoint:
      t=0  the path's own seed:                      0, 1, 2
      t=1  candidates zr+(0,d) ok, zr+(0,-2d) ok, zr+(0.3,0) fails; path 0 comes from
           zr+(0,0.25) -> nearest is seed 0, path 1 from zr-(0,0.25) -> seed 1,
           path 2 from zr -> seed 0 (d < 2d):       0, 1, 0
      t=2  seeds 1 and 2 identical and ok, seed 0 fails: tie to the lower: 1, 1, 1
      t=3  nothing ok; seed 1 non-finite; seeds 0, 2 at infinity distance 0.3 and 0.15
           from the common previous waypoint -> nearest finite:         2, 2, 2
      t=4  nothing finite: the previous waypoint again."""
    rb = oracle.Robot(L=[0.10], r=[0.010], u_max=[0.010])
    d = 2e-3
    zr = np.array([[0.2, 0.1], [0.2, 0.1], [0.4, 0.1], [0.5, 0.1], [0.3, 0.3]])
    cand = np.zeros((3, 5, 2))
    cand[:, 0] = zr[0] + np.array([[0, 0.25], [0, -0.25], [0, 0]])
    cand[:, 1] = zr[1] + np.array([[0, d], [0, -2 * d], [0.3, 0]])
    cand[:, 2] = zr[2] + np.array([[0.3, 0], [0, 0], [0, 0]])
    cand[:, 3] = zr[3] + np.array([[0, 0.3], [0, 0], [0, -0.15]])
    cand[1, 3] = np.nan
    cand[:, 4] = np.nan
    seeds = oracle.z_to_u(rb, cand.reshape(3, 5, 1, 2))
    _, fr = oracle.fk(rb, oracle.z_to_u(rb, zr.reshape(5, 1, 2)))
    z = oracle.path_seeds(rb, oracle.Weights(), oracle.Problem("path", fr[:, -1], H=4), oracle.Opts(), seeds, 0)
    src = [[0, 1, 2], [0, 1, 0], [1, 1, 1], [2, 2, 2]]
    for t in range(4):
        for s in range(3):
            assert np.abs(z[s, t, 0] - cand[src[t][s], t]).max() <= 1e-15, (s, t, z[s, t, 0])
    assert np.array_equal(z[:, 4], z[:, 3])
