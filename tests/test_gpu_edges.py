"""Edge cases of the path, trajectory and batch entry points: empty batches, a
single waypoint, the shortest trajectory, the longest horizon, the most spheres,
non-finite seeds, and batches with one problem or one kind."""
import numpy as np
import pytest

from helpers import aos, soa
from paper_2607_11340_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

L3, R3, B3 = [0.10, 0.08, 0.06], [0.010, 0.008, 0.006], 0.008


@pytest.fixture(scope="module")
def cr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_11340_amd import crsolver
    return crsolver


def rob(oracle, cr, K=4):
    return (oracle.Robot(L=L3, r=R3, u_max=[B3] * 3, pts_per_seg=K), cr.Robot(L=L3, r=R3, u_max=[B3] * 3, pts_per_seg=K))


def path_case(oracle, ro, rng, P, H, S):
    uref = I.smooth_actuation_paths(rng, 3, B3, P, H + 1)
    _, fr = oracle.fk(ro, uref)
    seeds = uref[:, None] + rng.normal(size=(P, S, H + 1, 3, 3)) * 4e-4
    return fr[:, :, -1], seeds


def test_empty_batches_return_ok(oracle, cr):
    _, rg = rob(oracle, cr)
    z = torch.zeros((12, 0), dtype=torch.float64, device="cuda")
    s = torch.zeros((9, 0), dtype=torch.float64, device="cuda")
    u, err, st = cr.solve_path(rg, z, s, 5)
    assert u.shape == (9, 0) and st.numel() == 0
    ends = torch.zeros((18, 0), dtype=torch.float64, device="cuda")
    u, err, st = cr.solve_traj(rg, ends, s, 5)
    assert st.numel() == 0


@pytest.mark.parametrize("H", [0, 1])
def test_path_with_one_or_two_waypoints_fp64(oracle, cr, H):
    """A path of a single waypoint is IK with the path solver's machinery; both
    horizons equal the oracle's FP64 plain solve."""
    print(f"path H={H}", flush=True)
    ro, rg = rob(oracle, cr)
    rng = np.random.default_rng(600 + H)
    P, S = 5, 3
    T, seeds = path_case(oracle, ro, rng, P, H, S)
    Tt = torch.tensor(soa(T, 2), device="cuda")
    us = torch.tensor(soa(seeds, 2), device="cuda")
    W = cr.Weights(w_vel=1e-2, w_acc=1e-2)
    u, err, st = cr.solve_path(rg, Tt, us, H, W, cr.Opts(n_final=0, k_init=4, k_final=0), dtype=torch.float64)
    u = aos(u.cpu().numpy(), (3, 3)).reshape(P, H + 1, 3, 3)
    st = st.cpu().numpy()
    for p in range(P):
        ref = oracle.solve(ro, oracle.Weights(w_vel=1e-2, w_acc=1e-2), oracle.Problem("path", T[p], H=H),
                           oracle.Opts(n_final=0, k_init=4, k_final=0), seeds[p])
        assert st[p] == ref["status"]
        assert np.abs(u[p] - ref["u"]).max() <= 1e-9 * B3


def test_longest_horizon_and_most_spheres(oracle, cr):
    """H = 255 (256 waypoints, four waves per trajectory) and 512 spheres (the
    largest allowed): FP64 iterates equal the oracle's; too large an LDS need is
    rejected with CR_EINVAL rather than launched."""
    print("longest horizon", flush=True)
    ro, rg = rob(oracle, cr, K=2)
    rng = np.random.default_rng(610)
    H, P, S = 255, 1, 1
    ends = I.uniform_actuation(rng, 3, B3, 2)
    seeds = I.perturbed_linear_paths(rng, ends[0], ends[1], 2, H + 1, B3)[1:][None]
    us = torch.tensor(soa(seeds, 2), device="cuda")
    e = torch.tensor(np.concatenate([ends[0].ravel(), ends[1].ravel()]).reshape(-1, 1), device="cuda")
    u, err, st = cr.solve_traj(rg, e, us, H, cr.Weights(), cr.Opts(n_final=0, k_init=2, k_final=0),
                               dtype=torch.float64)
    u = aos(u.cpu().numpy(), (3, 3)).reshape(H + 1, 3, 3)
    z0 = oracle.u_to_z(ro, seeds[0, 0]).ravel()
    zk, _, _, _, _ = oracle.lm(ro, oracle.Weights(), oracle.Problem("traj", (ends[0], ends[1]), H=H), oracle.Opts(),
                               z0, 1e-3, 2)
    assert np.abs(u - oracle.z_to_u(ro, zk.reshape(H + 1, 3, 2))).max() <= 1e-9 * B3
    # 512 spheres on a short horizon run; on the longest horizon they exceed the LDS budget
    sph = I.spheres(rng, 512, [0.5, 0.5, 0.5], [0.6, 0.6, 0.6], 0.005, 0.01)   # far away: no contact
    sp = (torch.tensor(np.ascontiguousarray(sph.T), device="cuda"), False, 512)
    H2 = 7
    seeds2 = I.perturbed_linear_paths(rng, ends[0], ends[1], 2, H2 + 1, B3)[1:][None]
    u2, _, st2 = cr.solve_traj(rg, e, torch.tensor(soa(seeds2, 2), device="cuda"), H2, cr.Weights(),
                               cr.Opts(n_final=0, k_init=2, k_final=0), dtype=torch.float64, spheres=sp)
    u3, _, _ = cr.solve_traj(rg, e, torch.tensor(soa(seeds2, 2), device="cuda"), H2, cr.Weights(),
                             cr.Opts(n_final=0, k_init=2, k_final=0), dtype=torch.float64)
    assert torch.equal(u2, u3)   # spheres out of reach change nothing
    with pytest.raises(cr.CRError) as ei:
        cr.solve_traj(rg, e, us, H, cr.Weights(), cr.Opts(n_final=0, k_init=1, k_final=0), dtype=torch.float64,
                      spheres=sp)
    assert ei.value.status == cr.CR_EINVAL


def test_nonfinite_trajectory_seeds(oracle, cr):
    """A seed trajectory with a NaN is never selected; a problem whose seeds are
    all non-finite reports CR_NONFINITE and NaN outputs, its neighbours solve."""
    print("nonfinite trajectory seeds", flush=True)
    ro, rg = rob(oracle, cr)
    rng = np.random.default_rng(620)
    P, S, H = 3, 4, 6
    T, seeds = path_case(oracle, ro, rng, P, H, S)
    seeds = seeds.copy()
    seeds[0, 1, 3, 1, 2] = np.nan       # one bad seed of problem 0
    seeds[1, :, 2, 0, 0] = np.inf       # every seed of problem 1
    u, err, st = cr.solve_path(rg, torch.tensor(soa(T, 2), device="cuda"), torch.tensor(soa(seeds, 2), device="cuda"),
                               H, cr.Weights(w_vel=1e-2, w_acc=1e-2), cr.Opts(n_final=2, k_init=30, k_final=10))
    st = st.cpu().numpy()
    u = u.cpu().numpy()
    assert st[1] == cr.NONFINITE and np.isnan(u[:, (H + 1):2 * (H + 1)]).all()
    assert st[0] == cr.SOLVED and st[2] == cr.SOLVED


def test_batch_of_one_problem_and_single_kind(oracle, cr):
    """One-problem batches of each kind equal the single-problem entry points;
    an IK-only batch equals cr_solve_ik problem by problem (FP64)."""
    print("batch of one", flush=True)
    ro, rg = rob(oracle, cr)
    rng = np.random.default_rng(630)
    ut = I.uniform_actuation(rng, 3, B3, 4)
    _, fr = oracle.fk(ro, ut)
    seeds = I.uniform_actuation(rng, 3, B3, 4 * 9).reshape(4, 9, 3, 3)
    probs = [dict(kind="ik", robot=0, H=0, task=fr[p, -1], seeds=seeds[p]) for p in range(4)]
    opts = [cr.Opts(n_final=2, k_init=6, k_final=3)] * 3
    W = [cr.Weights()] * 3
    for sub in (probs[:1], probs):
        batch = cr.Batch([rg], sub)
        u, err, st = cr.solve_batch(batch, W, opts, dtype=torch.float64)
        us = batch.unpack(u.cpu().numpy())
        T = torch.tensor(soa(fr[:len(sub), -1], 2), device="cuda")
        u1, _, s1 = cr.solve_ik(rg, T, torch.tensor(soa(seeds[:len(sub)], 2), device="cuda"), W[0], opts[0],
                                dtype=torch.float64)
        u1 = aos(u1.cpu().numpy(), (3, 3))
        for p in range(len(sub)):
            assert np.abs(us[p] - u1[p]).max() <= 1e-9 * B3
        assert np.array_equal(st.cpu().numpy(), s1.cpu().numpy())
