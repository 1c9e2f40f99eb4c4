"""Seeded synthetic inputs for CR-Solver workloads.

This module only draws random numbers and describes workload shapes.  It holds
none of the method's arithmetic (no kinematics, no cost, no solver), so both the
GPU library and the CPU oracle can be fed from it.  Every array is float64 and
item-major: actuations are ``[..., n, 3]`` tendon displacements in metres.

Poses that must be reachable (IK targets, path references) are made by the
caller from actuations drawn here, by running forward kinematics on its own side.

Recipes (the paper's benchmark sets are not available, so these stand in for
its 1000 uniformly sampled IK targets, its smooth reference paths and its random
sphere scenes; Sec. V-B, V-C, V-D):
  * uniform actuation: per segment u ~ U[-b, b]^3, minus its mean (tendon lengths
    of an inextensible segment sum to 3 L, eq. 4), accepted iff max |u| <= b;
  * smooth actuation path: per tendon a constant plus three Fourier harmonics with
    1/k amplitudes over the horizon, made zero-sum per segment and scaled so that
    max |u| <= 0.9 b;
  * spheres: centres uniform in a caller-given box, radii uniform in [r_lo, r_hi].
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 20260000

# Workload shapes.  Robot geometry in metres; b = bound on |tendon displacement|.
WORKLOADS = {
    "ik_plain_1seg": dict(
        kind="ik", L=[0.10], r=[0.010], b=0.010, P=16, S=64,
        k_init=100, k_final=0, n_final=0, K=10, dtype="f64", seed=BASE_SEED + 1),
    "ik_batched_3seg": dict(
        kind="ik", L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], b=0.008, P=4096, S=256,
        k_init=150, k_final=50, n_final=8, K=10, dtype="f32", seed=BASE_SEED + 2),
    "path_4seg": dict(
        kind="path", L=[0.08] * 4, r=[0.008] * 4, b=0.006, P=512, H=63, S=32,
        k_init=100, k_final=20, n_final=4, K=10, dtype="f32", seed=BASE_SEED + 3, k_seed=30,
        weights=dict(w_vel=1e-2, w_acc=1e-2)),
    "traj_5seg": dict(
        kind="traj", L=[0.06] * 5, r=[0.006] * 5, b=0.006, P=256, H=31, S=64, M=64,
        k_init=80, k_final=20, n_final=4, K=64, dtype="f32", seed=BASE_SEED + 4),
    # the trajectory workload with the PRM initializer of Algorithm 2 (Sec. V-C
    # compares it with the straight line): the same robot, horizon and seeds in
    # a random scene shaped like the paper's (27 spheres of radius 0.05 to 0.10
    # of the workspace's side: 25 to 50 mm for the ~0.5 m box of this robot's
    # tips); up to 8 of them sit on backbone points of the straight start-goal
    # motion; roadmaps of 1024 nodes with 10 neighbours, motions checked at 8
    # interior configurations
    "traj_prm_5seg": dict(
        kind="traj", L=[0.06] * 5, r=[0.006] * 5, b=0.006, P=256, H=31, S=64, M=27,
        k_init=80, k_final=20, n_final=4, K=64, dtype="f32", seed=BASE_SEED + 8, blockers=8, sph_r=(0.025, 0.05),
        prm=dict(n_nodes=1024, k=10, n_check=8, max_attempts=8)),
    # extendable robot among obstacles (Sec. V-B, the extendable row of Table II):
    # segment lengths free within [0.5, 1.5] of nominal, a 3 x 3 x 3 lattice of
    # spheres (radius 0.2 of a segment length, the paper's ratio) with seeded
    # jitter, targets kept only if their configuration clears the lattice
    "ik_ext_4seg": dict(
        kind="ik", L=[0.08] * 4, r=[0.008] * 4, b=0.006, L_min=[0.04] * 4, L_max=[0.12] * 4, P=1024, S=128,
        k_init=150, k_final=50, n_final=8, K=10, dtype="f32", seed=BASE_SEED + 6,
        lattice=dict(xy=(-0.15, 0.0, 0.15), z=(0.10, 0.22, 0.34), radius=0.016, jitter=0.01)),
    # the 3-segment robot among convex obstacles (the convex pieces of Sec. V's
    # scenes; synthetic boxes stand in for its shelves and cabinets): 12 oriented
    # boxes per problem, half extents U[1, 5] cm, centres in the workspace box,
    # kept only if they clear the target configuration by 3 mm
    "ik_box_3seg": dict(
        kind="ik", L=[0.10, 0.08, 0.06], r=[0.010, 0.008, 0.006], b=0.008, P=1024, S=128,
        k_init=150, k_final=50, n_final=8, K=10, dtype="f32", seed=BASE_SEED + 7,
        boxes=dict(count=12, lo=(-0.2, -0.2, 0.0), hi=(0.2, 0.2, 0.3), half_lo=0.01, half_hi=0.05, clear=3e-3)),
}


def line_blockers(rng: np.random.Generator, ends: np.ndarray, count: int, r_lo: float, r_hi: float, points,
                  body: np.ndarray, clear: float = 1e-3, rounds: int = 16):
    """Spheres [P, count, 4] in the way of each problem's straight motion between
    ends[p, 0] and ends[p, 1] ([P, 2, n, 3] actuations): a candidate is centred on
    a backbone point of the distal half of the configuration (1 - s) u_start +
    s u_goal, s ~ U[0.25, 0.75], radius U[r_lo, r_hi], and kept if it clears the
    start and goal backbones by `clear`; after `rounds` rounds of 4 * count
    candidates a problem keeps the blockers it has (start and goal too close for
    more).  points(u [B, n, 3]) -> [B, Q, 3] gives the caller's backbone points (Q
    per configuration, radii body [Q]).  Returns the spheres (rows past a
    problem's count are zero) and the count per problem [P]."""
    P = ends.shape[0]
    end_pts = points(ends.reshape((2 * P,) + ends.shape[2:])).reshape(P, -1, 3)
    out = np.zeros((P, count, 4))
    have = np.zeros(P, dtype=int)
    for _ in range(rounds):
        if (have >= count).all():
            break
        todo = np.flatnonzero(have < count)
        m = 4 * count
        s = rng.uniform(0.25, 0.75, size=(len(todo), m))
        u = (1.0 - s)[:, :, None, None] * ends[todo, 0][:, None] + s[:, :, None, None] * ends[todo, 1][:, None]
        pts = points(u.reshape((-1,) + ends.shape[2:])).reshape(len(todo), m, -1, 3)
        Q = pts.shape[2]
        idx = rng.integers(Q // 2, Q, size=(len(todo), m))
        rad = rng.uniform(r_lo, r_hi, size=(len(todo), m))
        for a, p in enumerate(todo):
            for c in range(m):
                if have[p] >= count:
                    break
                cen = pts[a, c, idx[a, c]]
                if (np.linalg.norm(end_pts[p] - cen, axis=1) - rad[a, c] - np.tile(body, 2)).min() > clear:
                    out[p, have[p]] = [*cen, rad[a, c]]
                    have[p] += 1
    return out, have


def random_boxes(rng: np.random.Generator, count: int, lo, hi, half_lo: float, half_hi: float):
    """`count` oriented boxes: centres [count, 3] uniform in [lo, hi], half extents
    [count, 3] uniform in [half_lo, half_hi], rotations [count, 3, 3] (the Q of a
    QR factorisation of a Gaussian matrix, columns the box axes)."""
    c = rng.uniform(np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64), size=(count, 3))
    h = rng.uniform(half_lo, half_hi, size=(count, 3))
    R = np.stack([np.linalg.qr(rng.normal(size=(3, 3)))[0] for _ in range(count)])
    return c, h, R


def box_halfspaces(c, h, R) -> np.ndarray:
    """The six half-spaces n.x <= d of a box (centre c, half extents h, axes the
    columns of R) as rows (nx, ny, nz, d)."""
    out = np.empty((6, 4))
    for k in range(3):
        for q, sgn in enumerate((1.0, -1.0)):
            n = sgn * R[:, k]
            out[2 * k + q, :3] = n
            out[2 * k + q, 3] = n @ c + h[k]
    return out


def extended_actuation(rng: np.random.Generator, n: int, b, e_lo, e_hi, count: int) -> np.ndarray:
    """`count` actuations [count, n, 3] of extensible segments: a uniform zero-sum
    bending part (as uniform_actuation) plus a common mode U[e_lo, e_hi] per segment
    (the change of the segment's length)."""
    e_lo = np.broadcast_to(np.asarray(e_lo, dtype=np.float64), (n,))
    e_hi = np.broadcast_to(np.asarray(e_hi, dtype=np.float64), (n,))
    bend = uniform_actuation(rng, n, b, count)
    return bend + rng.uniform(e_lo, e_hi, size=(count, n))[:, :, None]


def sphere_lattice(rng: np.random.Generator, xy, z, radius: float, jitter: float) -> np.ndarray:
    """A len(xy) x len(xy) x len(z) lattice of spheres [N, 4], each centre moved by
    U[-jitter, jitter] per axis."""
    c = np.array([[x, y, zz] for x in xy for y in xy for zz in z], dtype=np.float64)
    c = c + rng.uniform(-jitter, jitter, size=c.shape)
    return np.concatenate([c, np.full((len(c), 1), radius)], axis=1)


# Uneven batch: problem mix and ranges (robot geometry of path_4seg per segment;
# iteration budgets of the IK / path / trajectory workloads).
UNEVEN = dict(P=2048, frac=(0.60, 0.25, 0.15), n=(1, 6), H=(1, 64), S=(16, 512), M=(0, 64),
              L=0.08, r=0.008, b=0.006, K=10, seed=BASE_SEED + 5)


def uneven_problems(rng: np.random.Generator, P: int, spec: dict = None) -> list:
    """Shapes and random draws of an uneven batch: per problem a dict with kind
    ('ik' | 'path' | 'traj'), n, H (0 for IK), S, M and the actuations the caller
    turns into tasks (IK: u_true [n,3]; PATH: u_ref [H+1,n,3]; TRAJ: u_start,
    u_goal [n,3]), seeds [S, H+1, n, 3] and 4*M candidate spheres [4M, 4] (the
    caller keeps the first M that clear its configurations).  Path seeds are
    uniform IK seeds per (seed, waypoint) for the exploration stage; trajectory
    seeds are perturbed straight lines."""
    spec = spec or UNEVEN
    b = spec["b"]
    kinds = rng.choice(3, size=P, p=list(spec["frac"]))
    out = []
    for q in range(P):
        kind = ("ik", "path", "traj")[kinds[q]]
        n = int(rng.integers(spec["n"][0], spec["n"][1] + 1))
        H = 0 if kind == "ik" else int(rng.integers(spec["H"][0], spec["H"][1] + 1))
        S = int(rng.integers(spec["S"][0], spec["S"][1] + 1))
        M = int(rng.integers(spec["M"][0], spec["M"][1] + 1))
        Tn = H + 1
        d = dict(kind=kind, n=n, H=H, S=S, M=M)
        if kind == "ik":
            d["u_true"] = uniform_actuation(rng, n, b, 1)[0]
            d["seeds"] = uniform_actuation(rng, n, b, S).reshape(S, 1, n, 3)
        elif kind == "path":
            d["u_ref"] = smooth_actuation_paths(rng, n, b, 1, Tn)[0]
            d["seeds"] = uniform_actuation(rng, n, b, S * Tn).reshape(S, Tn, n, 3)
        else:
            ends = uniform_actuation(rng, n, b, 2)
            d["u_start"], d["u_goal"] = ends[0], ends[1]
            d["seeds"] = perturbed_linear_paths(rng, ends[0], ends[1], S, Tn, b)
        reach = n * spec["L"]
        d["sphere_pool"] = spheres(rng, 4 * M, [-0.7 * reach, -0.7 * reach, 0.0], [0.7 * reach, 0.7 * reach, reach],
                                   0.005, 0.02)
        out.append(d)
    return out


def rng_for(name: str, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(WORKLOADS[name]["seed"] * 1000 + salt))


def uniform_actuation(rng: np.random.Generator, n: int, b, count: int) -> np.ndarray:
    """`count` actuations [count, n, 3], each segment zero-sum with |u| <= b."""
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), (n,))
    out = np.empty((count, n, 3))
    for i in range(n):
        filled = 0
        while filled < count:
            m = max(16, int(1.2 * (count - filled)) + 16)
            x = rng.uniform(-b[i], b[i], size=(m, 3))
            x = x - x.mean(axis=1, keepdims=True)
            ok = x[np.abs(x).max(axis=1) <= b[i]]
            take = min(len(ok), count - filled)
            out[filled:filled + take, i] = ok[:take]
            filled += take
    return out


def smooth_actuation_paths(rng: np.random.Generator, n: int, b, count: int, T: int) -> np.ndarray:
    """`count` smooth actuation trajectories [count, T, n, 3] with max |u| <= 0.9 b."""
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), (n,))
    t = np.arange(T, dtype=np.float64) / max(T - 1, 1)
    out = np.empty((count, T, n, 3))
    for i in range(n):
        base = rng.uniform(-1.0, 1.0, size=(count, 1, 3))
        sig = np.repeat(base, T, axis=1)
        for k in (1, 2, 3):
            cc = rng.uniform(-1.0, 1.0, size=(count, 1, 3))
            ss = rng.uniform(-1.0, 1.0, size=(count, 1, 3))
            ang = 2.0 * np.pi * k * t[None, :, None]
            sig = sig + (cc * np.cos(ang) + ss * np.sin(ang)) / k
        sig = sig - sig.mean(axis=2, keepdims=True)
        peak = np.abs(sig).max(axis=(1, 2), keepdims=True)
        out[:, :, i, :] = sig * (0.9 * b[i] / np.maximum(peak, 1e-300))
    return out


def path_bumps(rng: np.random.Generator, n: int, count: int, T: int, b, amp: float = 0.5) -> np.ndarray:
    """Perturbations [count, T, n, 3] of trajectory seeds: bump 0 is zero, the
    others are two half-sine bumps per tendon of amplitude U[-amp, amp] * b over
    the horizon, made zero-sum per segment."""
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), (n,))
    s = np.arange(T, dtype=np.float64) / max(T - 1, 1)
    out = np.zeros((count, T, n, 3))
    for q in range(1, count):
        bump = np.zeros((T, n, 3))
        for k in (1, 2):
            c = rng.uniform(-amp, amp, size=(n, 3)) * b[:, None]
            bump += np.sin(np.pi * k * s)[:, None, None] * c[None]
        bump -= bump.mean(axis=2, keepdims=True)
        out[q] = bump
    return out


def perturbed_linear_paths(rng: np.random.Generator, u_start: np.ndarray, u_goal: np.ndarray,
                           count: int, T: int, b, amp: float = 0.5) -> np.ndarray:
    """Trajectory seeds [count, T, n, 3] between u_start and u_goal ([n, 3] each):
    seed 0 is the straight interpolation (the linear initializer of Sec. V-C),
    the others add path_bumps and are scaled per waypoint back inside |u| <= b."""
    n = u_start.shape[0]
    bumps = path_bumps(rng, n, count, T, b, amp)
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), (n,))
    s = np.arange(T, dtype=np.float64) / max(T - 1, 1)
    lin = (1.0 - s)[:, None, None] * u_start[None] + s[:, None, None] * u_goal[None]
    out = np.repeat(lin[None], count, axis=0)
    for q in range(1, count):
        x = out[q] + bumps[q]
        peak = np.abs(x).max(axis=2)  # [T, n]
        scale = np.minimum(1.0, b[None, :] / np.maximum(peak, 1e-300))
        out[q] = x * scale[:, :, None]
    return out


def spheres(rng: np.random.Generator, count: int, lo, hi, r_lo: float, r_hi: float) -> np.ndarray:
    """`count` spheres [count, 4] = (cx, cy, cz, radius), centres uniform in [lo, hi]^3."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    c = rng.uniform(lo, hi, size=(count, 3))
    r = rng.uniform(r_lo, r_hi, size=(count, 1))
    return np.concatenate([c, r], axis=1)
