"""Shared test helpers: layout conversion between the oracle (item-major numpy)
and the GPU library (structure-of-arrays torch), and seeded IK workloads whose
targets come from the oracle's forward kinematics."""
import numpy as np

from paper_2607_11340_amd import inputs as I


def soa(x: np.ndarray, comp_dims: int):
    """[batch..., comp...] -> [prod(comp), prod(batch)] contiguous float64."""
    lead = x.shape[: x.ndim - comp_dims]
    B = int(np.prod(lead)) if lead else 1
    return np.ascontiguousarray(x.reshape(B, -1).T)


def aos(x: np.ndarray, comp_shape):
    """[prod(comp), B] -> [B, comp...]."""
    return np.ascontiguousarray(x.T).reshape((x.shape[1],) + tuple(comp_shape))


def robots(O, cr, L, r, b, K=10, theta_max=np.pi):
    n = len(L)
    bb = list(np.broadcast_to(np.asarray(b, dtype=float), (n,)))
    return (O.Robot(L=list(L), r=list(r), u_max=bb, pts_per_seg=K, theta_max=theta_max),
            cr.Robot(L=list(L), r=list(r), u_max=bb, pts_per_seg=K, theta_max=theta_max))


def ik_workload(O, spec_name, P=None, S=None, salt=0):
    """(oracle robot, u_true [P,n,3], targets [P,3,4], seeds [P,S,n,3]) for a named IK workload."""
    spec = I.WORKLOADS[spec_name]
    P = P or spec["P"]
    S = S or spec["S"]
    rng = I.rng_for(spec_name, salt)
    n = len(spec["L"])
    rb = O.Robot(L=spec["L"], r=spec["r"], u_max=[spec["b"]] * n)
    u_true = I.uniform_actuation(rng, n, spec["b"], P)
    seeds = I.uniform_actuation(rng, n, spec["b"], P * S).reshape(P, S, n, 3)
    _, fr = O.fk(rb, u_true)
    return rb, u_true, fr[:, -1], seeds


def normwise_rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))
