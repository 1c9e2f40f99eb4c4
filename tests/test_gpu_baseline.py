"""The plain per-problem FP32 comparison solve (cr_baseline_solve_ik): the same
Algorithm 1 as cr_solve_ik built from separate kernels with a forward-mode
Jacobian.  FP32 throughout, so it is judged against the oracle at FP32-level
tolerance on a well-conditioned case and by solve quality on the headline shape."""
import numpy as np
import pytest

from helpers import aos, ik_workload, robots, soa
from paper_2607_11340_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_11340_amd import crsolver
    return crsolver


def _b0(cr, rg, T, seeds, opts):
    P, S = seeds.shape[:2]
    u, err, st = cr.baseline_solve_ik(rg, torch.tensor(soa(T, 2), device="cuda"),
                                      torch.tensor(soa(seeds, 2), device="cuda"), cr.Weights(), opts)
    torch.cuda.synchronize()
    return aos(u.cpu().numpy(), (rg.n, 3)), err.cpu().numpy().T, st.cpu().numpy()


@pytest.mark.parametrize("k", [1, 3])
def test_baseline_iterates_single_segment(oracle, cr, k):
    """Plain method, one seed: k FP32 iterations equal the oracle's FP64 iterates
    to FP32 accuracy (1e-5 of the bound) on the single-segment robot."""
    print(f"baseline iterates k={k}", flush=True)
    spec = I.WORKLOADS["ik_plain_1seg"]
    ro, _, T, seeds = ik_workload(oracle, "ik_plain_1seg", P=16, S=1, salt=k)
    _, rg = robots(oracle, cr, spec["L"], spec["r"], spec["b"])
    u, _, _ = _b0(cr, rg, T, seeds, cr.Opts(n_final=0, k_init=k, k_final=0))
    for p in range(16):
        z0 = oracle.u_to_z(ro, seeds[p, 0]).ravel()
        zk, _, _, _, _ = oracle.lm(ro, oracle.Weights(), oracle.Problem("ik", T[p]), oracle.Opts(), z0, 1e-3, k)
        uk = oracle.z_to_u(ro, zk.reshape(1, 2))
        assert np.abs(u[p] - uk).max() <= 1e-5 * spec["b"], (p, np.abs(u[p] - uk).max())


def test_baseline_two_stage_quality(oracle, cr):
    """Headline shape on 24 targets x 256 seeds, 150 + 50 iterations: >= 95 %
    success; reported errors equal the oracle's FP64 re-evaluation."""
    print("baseline two-stage quality", flush=True)
    spec = I.WORKLOADS["ik_batched_3seg"]
    ro, _, T, seeds = ik_workload(oracle, "ik_batched_3seg", P=24, salt=11)
    _, rg = robots(oracle, cr, spec["L"], spec["r"], spec["b"])
    u, err, st = _b0(cr, rg, T, seeds, cr.Opts(n_final=spec["n_final"], k_init=spec["k_init"],
                                               k_final=spec["k_final"]))
    assert (st == cr.SOLVED).mean() >= 0.95, st
    for p in range(24):
        pe = oracle.pose_error(ro, oracle.u_to_z(ro, u[p]), T[p])
        assert abs(err[p, 0] - pe[1]) < 1e-12 and abs(err[p, 1] - pe[2]) < 1e-9
