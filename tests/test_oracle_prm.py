"""Pins of the oracle's PRM exploration stage (Algorithm 2: ParallelSample,
ParallelConnect, ConnectToRoadmap, Dijkstra, ResampleLinear).

Each step is checked against something other than itself: the k nearest
neighbours against scipy's k-d tree, shortest paths against scipy's Dijkstra on
the same graph, motion checks against a sphere centred on a backbone point of
the configuration the check visits, ResampleLinear against a polyline whose
equal-arc-length points are known in closed form, and the whole query against
the straight-line initializer where the scene is empty."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra
from scipy.spatial import cKDTree

from paper_2607_11340_amd import inputs as I


def _robot(oracle, n=3, K=6):
    return oracle.Robot(L=[0.10, 0.08, 0.06, 0.06, 0.05][:n], r=[0.010, 0.008, 0.006, 0.006, 0.005][:n],
                        u_max=[0.008] * n, pts_per_seg=K)


def test_knn_matches_kdtree(oracle):
    ro = _robot(oracle)
    N, k = 60, 5
    rm = oracle.prm_roadmap(ro, 3, N, k, 0, (4, 5))
    x = rm["nodes"].reshape(N, -1)
    assert (rm["attempts"] == 1).all()
    _, idx = cKDTree(x).query(x, k=k + 1)
    for i in range(N):
        want = [j for j in idx[i] if j != i][:k]
        assert list(rm["nbr"][i]) == want, i
    # no checks: every listed motion is free, and the graph is their union
    for i in range(N):
        assert set(rm["adj"][i]) == set(rm["nbr"][i]) | {j for j in range(N) if i in rm["nbr"][j]}
        assert rm["adj"][i] == sorted(rm["adj"][i]) and i not in rm["adj"][i]
        for j, w in zip(rm["adj"][i], rm["adj_w"][i]):
            assert abs(w - np.linalg.norm(x[i] - x[j])) <= 1e-15 * w


def test_motion_check_visits_interior_configurations(oracle):
    """A sphere centred on the tip of the motion's midpoint configuration: one
    interior check (t = 1/2) lands on it, with clearance -R - r; two checks
    (t = 1/3, 2/3) pass beside it; no check sees nothing."""
    ro = _robot(oracle)
    rng = np.random.default_rng(2)
    ua, ub = I.uniform_actuation(rng, 3, 0.008, 2)
    _, _, pts = oracle.fk(ro, 0.5 * (ua + ub), points=True)
    R = 0.004
    sph = np.array([[*pts[-1, -1], R]])
    g1 = oracle.motion_gap(ro, ua, ub, 1, sph)
    assert abs(g1 - (-R - ro.r[2])) <= 1e-15
    want2 = min(oracle.config_gap(ro, ua + (ub - ua) / 3, sph), oracle.config_gap(ro, ua + 2 * (ub - ua) / 3, sph))
    assert abs(oracle.motion_gap(ro, ua, ub, 2, sph) - want2) <= 1e-12 and want2 > g1 + 1e-3
    assert oracle.motion_gap(ro, ua, ub, 0, sph) == np.inf
    # the clearance of one configuration in closed form: a straight robot's tip on
    # the z axis at height sum(L), a sphere on the axis above it
    straight = np.zeros((3, 3))
    top = sum(ro.L[:3])
    assert abs(oracle.config_gap(ro, straight, np.array([[0.0, 0.0, top + 0.05, 0.01]])) - (0.05 - 0.01 - 0.006)) \
        <= 1e-15


def _graph(rm, q, N):
    """Dense adjacency of the query graph (roadmap + start N + goal N + 1)."""
    W = np.zeros((N + 2, N + 2))
    for i in range(N):
        for j, w in zip(rm["adj"][i], rm["adj_w"][i]):
            W[i, j] = w
    nodes = rm["nodes"].reshape(N, -1)
    for end, lst in ((N, q["start_nbr"]), (N + 1, q["goal_nbr"])):
        for j in lst:
            if j >= 0:
                W[end, j] = W[j, end] = np.linalg.norm(nodes[j] - (q["qs"] if end == N else q["qg"]))
    if not q["direct_gap"] < 0:
        W[N, N + 1] = W[N + 1, N] = np.linalg.norm(q["qs"] - q["qg"])
    return W


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_shortest_path_matches_scipy(oracle, seed):
    """Spheres around the straight motion between start and goal: the query's
    path is a shortest path of the roadmap graph by scipy's Dijkstra."""
    ro = _robot(oracle, K=4)
    rng = np.random.default_rng(10 + seed)
    us, ug = I.uniform_actuation(rng, 3, 0.008, 2)
    sph = []
    for t in (0.35, 0.5, 0.65):
        _, _, pts = oracle.fk(ro, us + t * (ug - us), points=True)
        sph.append([*pts[-1, -2], 0.006])
    sph = np.array(sph)
    N, k, E = 48, 6, 3
    rm = oracle.prm_roadmap(ro, seed, N, k, E, (7, 7), spheres=sph)
    q = oracle.prm_query(ro, rm, k, E, us, ug, 12, spheres=sph)
    q["qs"], q["qg"] = us.ravel(), ug.ravel()
    W = _graph(rm, q, N)
    d = dijkstra(csr_matrix(W), directed=False, indices=N)
    path = q["path"]
    if np.isfinite(d[N + 1]):
        assert path[0] == N and path[-1] == N + 1 and q["n_path"] == len(path) - 2
        allu = np.concatenate([rm["nodes"].reshape(N, -1), us.ravel()[None], ug.ravel()[None]])
        length = sum(np.linalg.norm(allu[a] - allu[b]) for a, b in zip(path[:-1], path[1:]))
        assert all(W[a, b] > 0 for a, b in zip(path[:-1], path[1:]))
        assert abs(length - d[N + 1]) <= 1e-14 * d[N + 1]
    else:
        assert q["n_path"] == -1


def test_resample_linear_closed_form(oracle):
    pts = np.array([[0.0, 0.0], [3.0, 0.0], [3.0, 4.0]])
    out = oracle.resample_linear(pts, np.array([0.0, 3.0, 7.0]), 7)
    want = np.array([[0, 0], [1, 0], [2, 0], [3, 0], [3, 1], [3, 2], [3, 3], [3, 4]], dtype=float)
    assert np.abs(out - want).max() <= 1e-15
    # a zero-length segment is passed over
    out = oracle.resample_linear(np.array([[0.0], [2.0], [2.0], [4.0]]), np.array([0.0, 2.0, 2.0, 4.0]), 4)
    assert np.abs(out[:, 0] - [0, 1, 2, 3, 4]).max() <= 1e-15
    # H = 1: the two ends
    out = oracle.resample_linear(pts, np.array([0.0, 3.0, 7.0]), 1)
    assert np.array_equal(out, pts[[0, 2]])


def test_empty_scene_gives_the_linear_initializer(oracle):
    """Nothing to avoid: the direct motion is free and shorter than any detour,
    so the PRM seeds are the straight-line seeds with the same perturbations."""
    ro = _robot(oracle)
    rng = np.random.default_rng(4)
    us, ug = I.uniform_actuation(rng, 3, 0.008, 2)
    rm = oracle.prm_roadmap(ro, 0, 40, 4, 2, (1, 2))
    S, H = 6, 9
    lin = I.perturbed_linear_paths(np.random.default_rng(5), us, ug, S, H + 1, 0.008)
    bumps = I.path_bumps(np.random.default_rng(5), 3, S, H + 1, 0.008)
    for linear in (False, True):
        q = oracle.prm_query(ro, rm, 4, 2, us, ug, H, S=S, bumps=bumps, linear=linear)
        assert q["n_path"] == 0
        assert np.abs(q["seeds"] - lin).max() <= 1e-17
        assert np.abs(q["seeds"].sum(axis=3)).max() <= 1e-17
        assert (np.abs(q["seeds"]) <= 0.008 * (1 + 1e-15)).all()


def test_blocked_direct_motion_detours(oracle):
    ro = _robot(oracle, K=4)
    rng = np.random.default_rng(6)
    us, ug = I.uniform_actuation(rng, 3, 0.008, 2)
    _, _, pts = oracle.fk(ro, 0.5 * (us + ug), points=True)
    sph = np.array([[*pts[-1, -1], 0.008]])
    rm = oracle.prm_roadmap(ro, 1, 64, 8, 3, (3, 3), spheres=sph)
    q = oracle.prm_query(ro, rm, 8, 3, us, ug, 15, spheres=sph)
    assert q["direct_gap"] < 0 and q["n_path"] >= 1
    nodes = rm["nodes"].reshape(64, -1)
    allu = np.concatenate([nodes, us.ravel()[None], ug.ravel()[None]])
    for a, b in zip(q["path"][:-1], q["path"][1:]):
        # a roadmap motion starts at its lower-indexed node, a query motion at the query
        lo, hi = (min(a, b), max(a, b)) if max(a, b) < 64 else ((a, b) if a >= 64 else (b, a))
        assert not oracle.motion_gap(ro, allu[lo], allu[hi], 3, sph) < 0
    seeds = q["seeds"][0].reshape(16, -1)
    assert np.array_equal(seeds[0], us.ravel()) and np.array_equal(seeds[-1], ug.ravel())
    # equal arc length: consecutive waypoints are as far apart as the path's
    # length over H, except where a waypoint interval spans a path corner
    L = sum(np.linalg.norm(allu[a] - allu[b]) for a, b in zip(q["path"][:-1], q["path"][1:]))
    steps = np.linalg.norm(np.diff(seeds, axis=0), axis=1)
    assert steps.max() <= L / 15 * (1 + 1e-12)
    assert np.sum(np.abs(steps - L / 15) <= 1e-12 * L) >= 15 - q["n_path"]


def test_not_connected_falls_back_to_straight_line(oracle):
    ro = _robot(oracle)
    rng = np.random.default_rng(8)
    us, ug = I.uniform_actuation(rng, 3, 0.008, 2)
    sph = np.array([[0.0, 0.0, 0.0, 1.0]])        # engulfs every configuration
    rm = oracle.prm_roadmap(ro, 0, 16, 4, 2, (1, 1), max_attempts=2, spheres=sph)
    assert (rm["attempts"] == -2).all() and (rm["nbr"] == oracle.PRM_NONE).all()
    q = oracle.prm_query(ro, rm, 4, 2, us, ug, 5, spheres=sph)
    assert q["n_path"] == -1 and q["start_nbr"] == [] and q["direct_gap"] < 0
    t = np.arange(6)[:, None] / 5
    assert np.abs(q["seeds"][0].reshape(6, -1) - ((1 - t) * us.ravel() + t * ug.ravel())).max() <= 1e-17
