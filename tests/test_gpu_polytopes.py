"""Convex obstacles (polytopes in half-space form, clearance sd(x) - r_i with
sd(x) = max_f (n_f . x - d_f)) on the GPU against the CPU oracle: IK cost and
adjoint gradient (FP64 1e-9; FP32 1e-5 plus the derived FP32 hinge allowance,
helpers.fp32_hinge_slack), FP64 LM iterates (1e-9), the FP64 two-stage solve
(answers, status including CR_COLLISION and errors equal the oracle's), the FP32
two-stage solve's quality among boxes, and the argument checks."""
import numpy as np
import pytest

from helpers import aos, fp32_hinge_slack, soa
from paper_2607_11340_amd import inputs as I
from test_oracle_polytopes import box_planes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GEOM = dict(L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], u_max=[0.008] * 3)


@pytest.fixture(scope="module")
def cr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_11340_amd import crsolver
    return crsolver


def near_boxes(oracle, ro, rng, u, n_box, pad=2, reach=(-6e-4, 4e-4)):
    """n_box oriented boxes per configuration u [P, n, 3], each with a face just
    off (or just into) a random backbone point: [P, n_box, 6 + pad, 4]."""
    P = u.shape[0]
    out = np.zeros((P, n_box, 6 + pad, 4))
    for p in range(P):
        _, _, pts = oracle.fk(ro, u[p], points=True)
        for j in range(n_box):
            i, k = rng.integers(0, ro.n), rng.integers(0, ro.pts_per_seg)
            q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
            h = rng.uniform(0.008, 0.03, size=3)
            c = pts[i, k] + q[:, 0] * (h[0] + ro.r[i] + rng.uniform(*reach))
            out[p, j] = box_planes(c, h, q, pad=pad)
    return out


def gpu_planes(poly, td):
    P, NPO, F = poly.shape[:3]
    t = torch.tensor(np.ascontiguousarray(poly.reshape(P * NPO * F, 4).T), device="cuda", dtype=td)
    return (t, True, NPO, F)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_polytope_cost_grad_parity(oracle, cr, dtype):
    print(f"polytope cost_grad {dtype}", flush=True)
    rng = np.random.default_rng(1000)
    P, S, K = 13, 9, 6
    ro, rg = oracle.Robot(**GEOM, pts_per_seg=K), cr.Robot(**GEOM, pts_per_seg=K)
    ut = I.uniform_actuation(rng, 3, 0.008, P)
    _, fr = oracle.fk(ro, ut)
    u = I.uniform_actuation(rng, 3, 0.008, P * S).reshape(P, S, 3, 3)
    poly = near_boxes(oracle, ro, rng, u[:, 0], 4)
    T = fr[:, -1]
    if dtype == "f32":
        u, T, poly = (x.astype(np.float32).astype(np.float64) for x in (u, T, poly))
    W = oracle.Weights()
    co, go = np.zeros((P, S)), np.zeros_like(u)
    active = 0
    for p in range(P):
        pb = oracle.Problem("ik", T[p], polytopes=poly[p])
        for s in range(S):
            co[p, s], go[p, s] = oracle.cost(ro, W, pb, u[p, s], grad=True)
            active += co[p, s] > oracle.cost(ro, W, oracle.Problem("ik", T[p]), u[p, s]) * (1 + 1e-9)
    assert active >= P, active
    td = torch.float64 if dtype == "f64" else torch.float32
    pbg = cr.CostProblem(rg, "ik", P, S, 0, torch.tensor(soa(T, 2), device="cuda", dtype=td), cr.Weights(),
                         polytopes=gpu_planes(poly, td))
    cost, g = cr.cost_grad(pbg, torch.tensor(soa(u[:, :, None], 2), device="cuda", dtype=td))
    torch.cuda.synchronize()
    cg = cost.double().cpu().numpy().reshape(P, S)
    gg = aos(g.double().cpu().numpy(), (3, 3)).reshape(P, S, 3, 3)
    tol = 1e-9 if dtype == "f64" else 1e-5
    slack = np.zeros((P, S, 2))
    if dtype == "f32":
        for p in range(P):
            for s in range(S):
                slack[p, s] = fp32_hinge_slack(oracle, ro, W, u[p, s], poly=poly[p])
    gn = np.linalg.norm(go.reshape(P, S, -1), axis=2)
    eg = np.linalg.norm((gg - go).reshape(P, S, -1), axis=2)
    ec = np.abs(cg - co)
    print(f"  active {active}, max cost rel {(ec / co).max():.2e}, max grad rel {(eg / gn).max():.2e}", flush=True)
    assert (ec <= tol * co + slack[..., 0]).all()
    assert (eg <= tol * gn + slack[..., 1]).all()


def _ik(cr, rg, T, seeds, opts, dtype, poly):
    u, err, st = cr.solve_ik(rg, torch.tensor(soa(T, 2), device="cuda"), torch.tensor(soa(seeds, 2), device="cuda"),
                             cr.Weights(), opts, dtype=dtype, polytopes=gpu_planes(poly, torch.float64))
    torch.cuda.synchronize()
    return aos(u.cpu().numpy(), (rg.n, 3)), err.cpu().numpy().T, st.cpu().numpy()


@pytest.mark.parametrize("k", [1, 3])
def test_polytope_fp64_lm_iterates_match(oracle, cr, k):
    print(f"polytope fp64 iterates k={k}", flush=True)
    rng = np.random.default_rng(1010 + k)
    P, K = 24, 6
    ro, rg = oracle.Robot(**GEOM, pts_per_seg=K), cr.Robot(**GEOM, pts_per_seg=K)
    ut = I.uniform_actuation(rng, 3, 0.008, P)
    _, fr = oracle.fk(ro, ut)
    seeds = I.uniform_actuation(rng, 3, 0.008, P).reshape(P, 1, 3, 3)
    poly = near_boxes(oracle, ro, rng, seeds[:, 0], 3)
    ug, _, _ = _ik(cr, rg, fr[:, -1], seeds, cr.Opts(n_final=0, k_init=k, k_final=0), "f64", poly)
    for p in range(P):
        pb = oracle.Problem("ik", fr[p, -1], polytopes=poly[p])
        z0 = oracle.u_to_z(ro, seeds[p, 0]).ravel()
        zk, _, _, _, _ = oracle.lm(ro, oracle.Weights(), pb, oracle.Opts(), z0, 1e-3, k)
        uk = oracle.z_to_u(ro, zk.reshape(3, 2))
        assert np.abs(ug[p] - uk).max() <= 1e-9 * 0.008, (p, np.abs(ug[p] - uk).max())


def test_polytope_two_stage_fp64_matches_oracle_solve(oracle, cr):
    print("polytope two-stage fp64", flush=True)
    rng = np.random.default_rng(1020)
    P, S, K = 16, 8, 6
    ro, rg = oracle.Robot(**GEOM, pts_per_seg=K), cr.Robot(**GEOM, pts_per_seg=K)
    ut = I.uniform_actuation(rng, 3, 0.008, P)
    _, fr = oracle.fk(ro, ut)
    seeds = I.uniform_actuation(rng, 3, 0.008, P * S).reshape(P, S, 3, 3)
    poly = near_boxes(oracle, ro, rng, seeds[:, 0], 3)
    opts = dict(n_final=3, k_init=4, k_final=3)
    ug, err, st = _ik(cr, rg, fr[:, -1], seeds, cr.Opts(**opts), "f64", poly)
    ncoll = 0
    for p in range(P):
        ref = oracle.solve(ro, oracle.Weights(), oracle.Problem("ik", fr[p, -1], polytopes=poly[p]),
                           oracle.Opts(**opts), seeds[p])
        assert st[p] == ref["status"], (p, st[p], ref["status"])
        assert np.abs(ug[p] - ref["u"]).max() <= 1e-9 * 0.008, (p, np.abs(ug[p] - ref["u"]).max())
        assert np.allclose(err[p], ref["err"], rtol=1e-9, atol=1e-13)
        ncoll += bool(st[p] & cr.COLLISION)
    print(f"  answers in contact: {ncoll}", flush=True)


def test_polytope_two_stage_quality(oracle, cr):
    """FP32 stage 1 + FP64 stage 2 among 8 boxes per problem that keep 3 mm clear
    of the target's own configuration: >= 95 % solved, every solved answer clears
    every box by the oracle's geometry."""
    print("polytope two-stage quality", flush=True)
    rng = np.random.default_rng(1030)
    P, S, K, NB = 128, 64, 8, 8
    ro, rg = oracle.Robot(**GEOM, pts_per_seg=K), cr.Robot(**GEOM, pts_per_seg=K)
    ut = I.uniform_actuation(rng, 3, 0.008, P)
    _, fr, pts_t = oracle.fk(ro, ut, points=True)
    body = np.repeat(np.asarray(GEOM["r"]), K)
    poly = np.zeros((P, NB, 6, 4))
    for p in range(P):
        j = 0
        while j < NB:
            q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
            h = rng.uniform(0.01, 0.04, size=3)
            c = rng.uniform([-0.2, -0.2, 0.0], [0.2, 0.2, 0.3])
            pl = box_planes(c, h, q)
            sd = (pts_t[p].reshape(-1, 3) @ pl[:, :3].T - pl[None, :, 3]).max(axis=1)
            if (sd - body).min() > 3e-3:
                poly[p, j] = pl
                j += 1
    seeds = I.uniform_actuation(rng, 3, 0.008, P * S).reshape(P, S, 3, 3)
    ug, err, st = _ik(cr, rg, fr[:, -1], seeds, cr.Opts(n_final=8, k_init=150, k_final=50), "f32", poly)
    solved = st == cr.SOLVED
    print(f"  success {solved.mean():.3f}", flush=True)
    assert solved.mean() >= 0.95, np.unique(st, return_counts=True)
    for p in np.nonzero(solved)[0]:
        _, _, pts = oracle.fk(ro, ug[p], points=True)
        x = pts.reshape(-1, 3)
        for pl in poly[p]:
            assert ((x @ pl[:, :3].T - pl[None, :, 3]).max(axis=1) - body).min() >= 0.0


def test_polytope_argument_checks(cr):
    rg = cr.Robot(**GEOM, pts_per_seg=4)
    poly = np.tile(box_planes(np.array([0.1, 0.0, 0.1]), np.array([0.01, 0.01, 0.01]))[None, None], (2, 1, 1, 1))
    seeds = torch.zeros((9, 2 * 4), dtype=torch.float64, device="cuda")
    T = torch.zeros((12, 2), dtype=torch.float64, device="cuda")
    ext = cr.Robot(**GEOM, pts_per_seg=4, L_min=[0.05] * 3, L_max=[0.12] * 3)
    with pytest.raises(cr.CRError):
        cr.solve_ik(ext, T, seeds, polytopes=gpu_planes(poly, torch.float64))
    bad = (gpu_planes(poly, torch.float64)[0], True, 1, 40)        # 40 planes per polytope
    with pytest.raises(cr.CRError):
        cr.solve_ik(rg, T, seeds, polytopes=bad)
    pbg = cr.CostProblem(rg, "path", 2, 1, 3, torch.zeros((12, 8), device="cuda", dtype=torch.float64), cr.Weights(),
                         polytopes=gpu_planes(poly, torch.float64))
    with pytest.raises(cr.CRError):
        cr.cost_grad(pbg, torch.zeros((9, 8), device="cuda", dtype=torch.float64))
