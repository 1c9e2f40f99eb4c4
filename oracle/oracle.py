"""Python access to the plain FP64 CPU oracle in ``oracle/cro.c``.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously correct reference
that the GPU library is checked against; only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code
with the GPU library (``paper_2607_11340_amd``) and never imports it.

Arrays are numpy float64, item-major:
  u  [..., n, 3]   tendon displacements (Sec. III-B, eq. 4 minus L_i)
  z  [..., n, c]   coordinates: bending (a, b) = theta (cos phi, sin phi), and for
                   extensible robots (c = 3) the extension e = mean tendon displacement
  T  [..., 3, 4]   pose [R | p]
"""
from __future__ import annotations

import ctypes as C
import heapq
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cro.c")
HDR = os.path.join(HERE, "cro.h")
LIB = os.path.join(HERE, "libcro.so")
MAX_SEG = 6
KIND = {"ik": 0, "path": 1, "traj": 2}
SOLVED, LIMIT_VIOLATION, COLLISION, NONFINITE, NOT_CONVERGED = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(HDR)):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Robot(C.Structure):
    _fields_ = [("n_seg", C.c_int32), ("pts_per_seg", C.c_int32),
                ("L", C.c_double * MAX_SEG), ("r", C.c_double * MAX_SEG),
                ("u_max", C.c_double * MAX_SEG), ("theta_max", C.c_double),
                ("extensible", C.c_int32), ("L_min", C.c_double * MAX_SEG), ("L_max", C.c_double * MAX_SEG),
                ("self_collision", C.c_int32)]


class _Weights(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "w_pos", "w_rot", "rho_lim", "rho_curv", "rho_coll", "margin", "rho_eq",
        "w_len", "w_vel", "w_acc", "v_max", "a_max", "dt")]


class _Opts(C.Structure):
    _fields_ = [("n_final", C.c_int32), ("k_init", C.c_int32), ("k_final", C.c_int32),
                ("ls_max", C.c_int32), ("lambda0", C.c_double), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("dup_eps", C.c_double), ("k_seed", C.c_int32)]


class _Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("H", C.c_int32), ("task", C.POINTER(C.c_double)),
                ("n_sph", C.c_int32), ("sph", C.POINTER(C.c_double)),
                ("n_poly", C.c_int32), ("n_planes", C.c_int32), ("planes", C.POINTER(C.c_double))]


@dataclass
class Robot:
    L: list
    r: list
    u_max: list
    pts_per_seg: int = 10
    theta_max: float = np.pi
    L_min: list = None     # extensible robots: bounds on each segment length (m);
    L_max: list = None     # both given <=> the segment lengths are decision variables
    self_collision: bool = False   # contact between non-adjacent segments counts (eq. 10)

    @property
    def n(self) -> int:
        return len(self.L)

    @property
    def extensible(self) -> bool:
        return self.L_min is not None and self.L_max is not None

    @property
    def nc(self) -> int:
        """coordinates per segment"""
        return 3 if self.extensible else 2

    def c(self) -> _Robot:
        s = _Robot()
        s.n_seg = self.n
        s.pts_per_seg = self.pts_per_seg
        for i in range(self.n):
            s.L[i], s.r[i], s.u_max[i] = self.L[i], self.r[i], self.u_max[i]
        s.theta_max = self.theta_max
        s.extensible = 1 if self.extensible else 0
        if self.extensible:
            for i in range(self.n):
                s.L_min[i], s.L_max[i] = self.L_min[i], self.L_max[i]
        s.self_collision = 1 if self.self_collision else 0
        return s


@dataclass
class Weights:
    w_pos: float = 1.0
    w_rot: float = 1.0
    rho_lim: float = 1e6
    rho_curv: float = 1e2
    rho_coll: float = 1e6
    margin: float = 1e-3
    rho_eq: float = 1e4
    w_len: float = 1.0
    w_vel: float = 1.0
    w_acc: float = 1.0
    v_max: float = float("inf")
    a_max: float = float("inf")
    dt: float = 1.0

    def c(self) -> _Weights:
        return _Weights(*[float(getattr(self, k)) for k, _ in _Weights._fields_])


@dataclass
class Opts:
    n_final: int = 8
    k_init: int = 150
    k_final: int = 50
    ls_max: int = 4
    lambda0: float = 1e-3
    lambda_min: float = 1e-12
    lambda_max: float = 1e12
    dup_eps: float = 1e-3
    k_seed: int = 0

    def c(self) -> _Opts:
        return _Opts(self.n_final, self.k_init, self.k_final, self.ls_max, self.lambda0,
                     self.lambda_min, self.lambda_max, self.dup_eps, self.k_seed)


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        R, W, O, P = C.POINTER(_Robot), C.POINTER(_Weights), C.POINTER(_Opts), C.POINTER(_Problem)
        L.cro_u_to_z.argtypes = [R, dp, dp]
        L.cro_z_to_u.argtypes = [R, dp, dp]
        L.cro_fk.argtypes = [R, dp, dp, dp, dp]
        L.cro_fk.restype = C.c_int
        L.cro_cost.argtypes = [R, W, P, dp, dp]
        L.cro_cost.restype = C.c_double
        L.cro_residuals.argtypes = [R, W, P, dp, dp, dp, C.c_int]
        L.cro_residuals.restype = C.c_int
        L.cro_pose_error.argtypes = [R, dp, dp, dp]
        L.cro_lm.argtypes = [R, W, P, O, dp, dp, C.c_int, dp, C.POINTER(C.c_int)]
        L.cro_lm.restype = C.c_int
        L.cro_chol_solve.argtypes = [C.c_int, C.c_int, dp, dp]
        L.cro_chol_solve.restype = C.c_int
        L.cro_select_top.argtypes = [C.c_int, C.c_int, dp, dp, dp, ip, C.c_int, C.c_double, ip]
        L.cro_solve.argtypes = [R, W, P, O, C.c_int, dp, dp, dp, ip, ip, dp]
        L.cro_path_seeds.argtypes = [R, W, P, O, C.c_int, dp, C.c_int, dp]
        L.cro_path_seeds.restype = None
        L.cro_solve.restype = C.c_int
        u64p = C.POINTER(C.c_uint64)
        L.cro_philox4x64.argtypes = [u64p, u64p, u64p]
        L.cro_philox4x64.restype = None
        L.cro_sample_seed.argtypes = [R, dp, C.c_int, u64p, C.c_int64, C.c_int32, C.c_int32, dp]
        L.cro_sample_seed.restype = C.c_int32
        L.cro_contact_gap.argtypes = [R, dp, C.c_int, dp]
        L.cro_contact_gap.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


class Problem:
    """One task instance: kind 'ik' (task T[3,4]), 'path' (T[H+1,3,4]) or
    'traj' (u_start[n,3], u_goal[n,3]); optional spheres [M,4]."""

    def __init__(self, kind: str, task, H: int = 0, spheres=None, polytopes=None):
        """polytopes: None or [n_poly, n_planes, 4] half-spaces (unit normal, offset)
        n.x <= d of convex obstacles."""
        self.kind, self.H = kind, int(H)
        if kind == "traj":
            us, ug = task
            self._task, p = _d(np.concatenate([np.ravel(us), np.ravel(ug)]))
        else:
            self._task, p = _d(np.ravel(task))
        sph = np.zeros((0, 4)) if spheres is None else np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
        self._sph, sp = _d(sph if len(sph) else np.zeros((1, 4)))
        pl = np.zeros((0, 1, 4)) if polytopes is None else np.asarray(polytopes, dtype=np.float64)
        self._pl, pp = _d(pl if pl.size else np.zeros((1, 1, 4)))
        self.c = _Problem(KIND[kind], self.H, p, len(sph), sp, len(pl), pl.shape[1] if len(pl) else 0, pp)


def u_to_z(robot: Robot, u):
    u = np.asarray(u, dtype=np.float64)
    flat = u.reshape(-1, robot.n * 3)
    nc = robot.nc
    out = np.empty((flat.shape[0], robot.n * nc))
    rc = robot.c()
    for k in range(flat.shape[0]):
        a, pa = _d(flat[k])
        o = np.empty(robot.n * nc)
        lib().cro_u_to_z(C.byref(rc), pa, o.ctypes.data_as(C.POINTER(C.c_double)))
        out[k] = o
    return out.reshape(u.shape[:-2] + (robot.n, nc))


def z_to_u(robot: Robot, z):
    z = np.asarray(z, dtype=np.float64)
    flat = z.reshape(-1, robot.n * robot.nc)
    out = np.empty((flat.shape[0], robot.n * 3))
    rc = robot.c()
    for k in range(flat.shape[0]):
        a, pa = _d(flat[k])
        o = np.empty(robot.n * 3)
        lib().cro_z_to_u(C.byref(rc), pa, o.ctypes.data_as(C.POINTER(C.c_double)))
        out[k] = o
    return out.reshape(z.shape[:-2] + (robot.n, 3))


def fk(robot: Robot, u, points: bool = False):
    """Returns arc [..., n, 3] (kappa, phi, L), frames [..., n, 3, 4] and optionally
    backbone points [..., n, K, 3]."""
    u = np.asarray(u, dtype=np.float64)
    lead = u.shape[:-2]
    flat = u.reshape(-1, robot.n * 3)
    B, n, K = flat.shape[0], robot.n, robot.pts_per_seg
    arc = np.empty((B, n * 3))
    frames = np.empty((B, n * 12))
    pts = np.empty((B, n * K * 3)) if points else None
    rc = robot.c()
    dp = C.POINTER(C.c_double)
    for k in range(B):
        a, pa = _d(flat[k])
        o1, o2 = np.empty(n * 3), np.empty(n * 12)
        o3 = np.empty(max(n * K * 3, 1))
        lib().cro_fk(C.byref(rc), pa, o1.ctypes.data_as(dp), o2.ctypes.data_as(dp),
                     o3.ctypes.data_as(dp) if points else None)
        arc[k], frames[k] = o1, o2
        if points:
            pts[k] = o3[: n * K * 3]
    out = (arc.reshape(lead + (n, 3)), frames.reshape(lead + (n, 3, 4)))
    if points:
        out = out + (pts.reshape(lead + (n, K, 3)),)
    return out


def cost(robot: Robot, weights: Weights, prob: Problem, u, grad: bool = False):
    """Penalised cost (eq. 17) of one seed, u [H+1, n, 3] (or [n, 3] for IK);
    returns cost or (cost, dC/du)."""
    u, pu = _d(u)
    g = np.empty_like(u) if grad else None
    rc, wc = robot.c(), weights.c()
    c = lib().cro_cost(C.byref(rc), C.byref(wc), C.byref(prob.c), pu,
                       g.ctypes.data_as(C.POINTER(C.c_double)) if grad else None)
    return (c, g) if grad else c


def residuals(robot: Robot, weights: Weights, prob: Problem, z, cap: int = 200000):
    """Residual vector r [m] and dense Jacobian J [m, N] at z."""
    z, pz = _d(z)
    N = z.size
    cap = min(cap, max(1, 2 ** 27 // max(N, 1)))
    r = np.empty(cap)
    J = np.empty((cap, N))
    rc, wc = robot.c(), weights.c()
    dp = C.POINTER(C.c_double)
    m = lib().cro_residuals(C.byref(rc), C.byref(wc), C.byref(prob.c), pz, r.ctypes.data_as(dp),
                            J.ctypes.data_as(dp), cap)
    if m < 0:
        raise ValueError("residual capacity exceeded")
    return r[:m].copy(), J[:m].copy()


def pose_error(robot: Robot, z, T):
    """(e, position error, rotation angle) of z [n, c] against T [3, 4] (eq. 18)."""
    z, pz = _d(z)
    T, pT = _d(T)
    out = np.empty(3)
    rc = robot.c()
    lib().cro_pose_error(C.byref(rc), pz, pT, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def lm(robot: Robot, weights: Weights, prob: Problem, opts: Opts, z, lam: float, iters: int):
    """Run `iters` LM iterations from z; returns (z, lambda, cost, failed, trials)."""
    z = np.array(z, dtype=np.float64, copy=True)
    pz = z.ctypes.data_as(C.POINTER(C.c_double))
    lamc = C.c_double(lam)
    costc = C.c_double(0.0)
    trials = C.c_int(0)
    rc, wc, oc = robot.c(), weights.c(), opts.c()
    failed = lib().cro_lm(C.byref(rc), C.byref(wc), C.byref(prob.c), C.byref(oc), pz, C.byref(lamc),
                          int(iters), C.byref(costc), C.byref(trials))
    return z, lamc.value, costc.value, bool(failed), trials.value


def chol_solve(M, y, bw=None):
    M = np.array(M, dtype=np.float64, copy=True)
    N = M.shape[0]
    x = np.array(y, dtype=np.float64, copy=True)
    rc = lib().cro_chol_solve(N, N - 1 if bw is None else int(bw), M.ctypes.data_as(C.POINTER(C.c_double)),
                              x.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise np.linalg.LinAlgError("not positive definite")
    return x, np.tril(M)


def select_top(z, e, pen, failed, n_final: int, dup_eps: float = 1e-3):
    z = np.asarray(z, dtype=np.float64)
    S = z.shape[0]
    z2, pz = _d(z.reshape(S, -1))
    e2, pe = _d(e)
    p2, pp = _d(pen)
    f2, pf = _i(np.zeros(S) if failed is None else failed)
    out = np.empty(n_final, dtype=np.int32)
    lib().cro_select_top(S, z2.shape[1], pz, pe, pp, pf, n_final, dup_eps,
                         out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out


def path_seeds(robot: Robot, weights: Weights, prob: Problem, opts: Opts, u_seed, k: int):
    """Per-waypoint IK and path assembly (cro_path_seeds); u_seed [S, H+1, n, 3]
    -> z [S, H+1, n, c]."""
    u_seed = np.asarray(u_seed, dtype=np.float64)
    S = u_seed.shape[0]
    us, pu = _d(u_seed)
    z = np.empty((S, prob.H + 1, robot.n, robot.nc))
    rc, wc, oc = robot.c(), weights.c(), opts.c()
    lib().cro_path_seeds(C.byref(rc), C.byref(wc), C.byref(prob.c), C.byref(oc), S, pu, int(k),
                         z.ctypes.data_as(C.POINTER(C.c_double)))
    return z


def solve(robot: Robot, weights: Weights, prob: Problem, opts: Opts, u_seed):
    """Two-stage solve of one problem from seeds u_seed [S, H+1, n, 3] (or [S, n, 3]).
    Returns dict(u, err(pos, rot), status, best, cost)."""
    u_seed = np.asarray(u_seed, dtype=np.float64)
    S = u_seed.shape[0]
    us, pu = _d(u_seed)
    T = prob.H + 1
    u_out = np.empty(T * robot.n * 3)
    err = np.empty(2)
    st = C.c_int32(0)
    best = C.c_int32(0)
    bc = C.c_double(0.0)
    rc, wc, oc = robot.c(), weights.c(), opts.c()
    dp = C.POINTER(C.c_double)
    r = lib().cro_solve(C.byref(rc), C.byref(wc), C.byref(prob.c), C.byref(oc), S, pu,
                        u_out.ctypes.data_as(dp), err.ctypes.data_as(dp), C.byref(st), C.byref(best),
                        C.byref(bc))
    if r != 0:
        raise ValueError("bad solve arguments")
    shape = (robot.n, 3) if prob.kind == "ik" else (T, robot.n, 3)
    return dict(u=u_out.reshape(shape), err=err, status=st.value, best=best.value, cost=bc.value)


def philox4x64(ctr, key):
    """Philox4x64-10 block: four uint64 words for counter ctr[4] under key[2]."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    u64p = C.POINTER(C.c_uint64)
    lib().cro_philox4x64(c.ctypes.data_as(u64p), k.ctypes.data_as(u64p), out.ctypes.data_as(u64p))
    return out


def sample_seeds(robot: Robot, P: int, S: int, key, max_attempts: int = 8, spheres=None):
    """SampleSeeds (Algorithm 1) for P problems x S seeds: u [P, S, n, 3] and the
    attempts per seed [P, S] (negative: still colliding after max_attempts).
    spheres: None, [M, 4] shared, or [P, M, 4] per problem."""
    n = robot.n
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    u64p = C.POINTER(C.c_uint64)
    rc = robot.c()
    u = np.zeros((P, S, n, 3))
    tries = np.zeros((P, S), dtype=np.int32)
    for p in range(P):
        sp = None if spheres is None else np.asarray(spheres, dtype=np.float64)
        if sp is not None and sp.ndim == 3:
            sp = sp[p]
        M = 0 if sp is None else len(sp)
        sarr, sptr = _d(sp if M else np.zeros((1, 4)))
        for s in range(S):
            out, po = _d(np.zeros(3 * n))
            tries[p, s] = lib().cro_sample_seed(C.byref(rc), sptr, M, k.ctypes.data_as(u64p), p, s,
                                                int(max_attempts), po)
            u[p, s] = out.reshape(n, 3)
    return u, tries


# ---------------------------------------------------------------------------
# PRM exploration stage of trajectory planning (Algorithm 2; Sec. IV-B).
#
# Readings, where the algorithm leaves the details open:
#  * configurations are tendon displacements u (3n numbers, zero-sum per
#    segment); the distance of two configurations is the Euclidean norm of their
#    difference, its square summed in component order;
#  * ParallelSample(N): node j of problem p is SampleSeeds' draw (key, p, j);
#    a node that still collides after max_attempts is discarded (kept in the
#    arrays, flagged by its negative attempt count);
#  * a straight motion from a to b is free iff each of its n_check interior
#    configurations a + t_m (b - a), t_m = m / (n_check + 1), m = 1..n_check,
#    clears the scene (SampleSeeds' test, margin 0); a roadmap motion starts at
#    the lower-indexed node, a query motion at the query configuration;
#  * ParallelConnect(V, k): each kept node lists its k nearest kept nodes
#    (ties to the lower index); the graph is undirected, {i, j} is an edge when
#    either lists the other with a free motion, weighted by their distance;
#  * ConnectToRoadmap(q): the k nearest kept nodes of q joined by free motions;
#    the direct start-goal motion is an edge too when it is free;
#  * Dijkstra: nodes 0..N-1 are the roadmap, N the start and N+1 the goal; nodes
#    settle in order of (distance, index), a relaxation needs a strictly
#    smaller distance, and the search ends when the goal settles;
#  * ResampleLinear(Q_path, H): waypoint t lies at arc length s_m t / H along the
#    path's polyline (s_i = distance of the i-th path node from the start), by
#    linear interpolation in the first segment whose end reaches it; waypoint 0
#    is the start and waypoint H the goal;
#  * start and goal not connected: the straight line between them;
#  * seeds for ParallelOptimize: seed 0 is Q'; seed s >= 1 adds the caller's
#    perturbation of that seed and scales each (waypoint, segment) back into
#    |u| <= u_max.
# ---------------------------------------------------------------------------
PRM_NONE = -(2 ** 31)


def config_gap(robot: Robot, u, spheres=None) -> float:
    """Smallest clearance of one configuration u [n, 3] (negative: collides)."""
    sph = np.zeros((0, 4)) if spheres is None else np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
    sarr, sp = _d(sph if len(sph) else np.zeros((1, 4)))
    ua, up = _d(np.ravel(u))
    rc = robot.c()
    return float(lib().cro_contact_gap(C.byref(rc), sp, len(sph), up))


def dist2(a, b):
    """Squared distance of configurations a [..., 3n] and b [..., 3n], summed in
    component order (broadcasting over leading axes)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.zeros(np.broadcast_shapes(a.shape[:-1], b.shape[:-1]))
    for c in range(a.shape[-1]):
        d = a[..., c] - b[..., c]
        out = out + d * d
    return out


def motion_gap(robot: Robot, ua, ub, n_check: int, spheres=None) -> float:
    """Smallest clearance over the interior configurations of the straight motion
    ua -> ub ([3n] each); INFINITY when n_check is 0 or nothing is in the way."""
    ua = np.ravel(np.asarray(ua, dtype=np.float64))
    ub = np.ravel(np.asarray(ub, dtype=np.float64))
    g = np.inf
    for m in range(1, n_check + 1):
        t = m / (n_check + 1)
        g = min(g, config_gap(robot, ua + t * (ub - ua), spheres))
    return g


def prm_roadmap(robot: Robot, p: int, N: int, k: int, n_check: int, key, max_attempts: int = 8, spheres=None):
    """ParallelSample(N) and ParallelConnect(V, k) for problem p's scene.

    Returns dict with
      nodes [N, n, 3], attempts [N] (negative: discarded),
      nbr [N, k] int: slot c of node i holds j (free motion), -1 - j (the motion
        collides) or PRM_NONE (fewer than k kept neighbours, or i discarded),
      gap [N, k]: smallest clearance over the slot's motion (INFINITY if none),
      adj: list of N sorted neighbour lists of the undirected graph,
      adj_w: their weights (distances)."""
    n = robot.n
    kk = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    u64p = C.POINTER(C.c_uint64)
    rc = robot.c()
    sph = None if spheres is None else np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
    M = 0 if sph is None else len(sph)
    sarr, sptr = _d(sph if M else np.zeros((1, 4)))
    nodes = np.zeros((N, 3 * n))
    att = np.zeros(N, dtype=np.int64)
    for j in range(N):
        out, po = _d(np.zeros(3 * n))
        att[j] = lib().cro_sample_seed(C.byref(rc), sptr, M, kk.ctypes.data_as(u64p), p, j, int(max_attempts), po)
        nodes[j] = out
    kept = att > 0
    nbr = np.full((N, k), PRM_NONE, dtype=np.int64)
    gap = np.full((N, k), np.inf)
    for i in range(N):
        if not kept[i]:
            continue
        d2 = dist2(nodes[i][None], nodes)
        order = [j for j in np.lexsort((np.arange(N), d2)) if j != i and kept[j]][:k]
        for c, j in enumerate(order):
            a, b = min(i, j), max(i, j)
            g = motion_gap(robot, nodes[a], nodes[b], n_check, sph)
            gap[i, c] = g
            nbr[i, c] = j if not g < 0.0 else -1 - j
    nb = [set() for _ in range(N)]
    for i in range(N):
        for j in nbr[i]:
            if j >= 0:
                nb[i].add(int(j))
                nb[int(j)].add(i)
    adj = [sorted(s) for s in nb]
    adj_w = [[float(np.sqrt(dist2(nodes[i], nodes[j]))) for j in adj[i]] for i in range(N)]
    return dict(nodes=nodes.reshape(N, n, 3), attempts=att, nbr=nbr, gap=gap, adj=adj, adj_w=adj_w)


def resample_linear(path_u, s, H: int):
    """ResampleLinear: H + 1 waypoints [H+1, 3n] at equal arc length along the
    polyline through path_u [m+1, 3n] whose cumulative lengths are s [m+1]."""
    path_u = np.asarray(path_u, dtype=np.float64)
    m = len(path_u) - 1
    out = np.empty((H + 1, path_u.shape[1]))
    out[0] = path_u[0]
    out[H] = path_u[m]
    for t in range(1, H):
        sig = s[m] * t / H
        i = 1
        while i < m and not sig <= s[i]:
            i += 1
        den = s[i] - s[i - 1]
        lam = (sig - s[i - 1]) / den if den != 0.0 else 0.0
        out[t] = path_u[i - 1] + lam * (path_u[i] - path_u[i - 1])
    return out


def prm_query(robot: Robot, rm: dict, k: int, n_check: int, u_start, u_goal, H: int, S: int = 1, bumps=None,
              spheres=None, linear: bool = False):
    """ConnectToRoadmap, Dijkstra and ResampleLinear for one query on roadmap rm
    (as prm_roadmap returns), then the S seeds of ParallelOptimize.

    bumps: None or [S, H+1, n, 3] perturbations (seed 0's is ignored).
    linear: skip the roadmap (the straight-line initializer).
    Returns dict with path (node indices, start N ... goal N+1), n_path (roadmap
    nodes on the path; -1: not connected, straight line), seeds [S, H+1, n, 3],
    the connections of both ends (start_nbr/goal_nbr: j or -1 - j as nbr) with
    their clearances, and the direct motion's clearance."""
    n = robot.n
    sph = None if spheres is None else np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
    qs = np.ravel(np.asarray(u_start, dtype=np.float64))
    qg = np.ravel(np.asarray(u_goal, dtype=np.float64))
    out = dict()
    if linear:
        path, n_path, pts, s = [None, None], 0, np.stack([qs, qg]), np.array([0.0, np.sqrt(dist2(qs, qg))])
    else:
        nodes = rm["nodes"].reshape(-1, 3 * n)
        N = len(nodes)
        kept = rm["attempts"] > 0
        ends = []
        for q in (qs, qg):
            d2 = dist2(q[None], nodes)
            order = [j for j in np.lexsort((np.arange(N), d2)) if kept[j]][:k]
            lst = []
            for j in order:
                g = motion_gap(robot, q, nodes[j], n_check, sph)
                lst.append((int(j), g, float(np.sqrt(d2[j]))))
            ends.append(lst)
        g_direct = motion_gap(robot, qs, qg, n_check, sph)
        out.update(start_nbr=[j if not g < 0.0 else -1 - j for j, g, _ in ends[0]],
                   goal_nbr=[j if not g < 0.0 else -1 - j for j, g, _ in ends[1]],
                   start_gap=[g for _, g, _ in ends[0]], goal_gap=[g for _, g, _ in ends[1]], direct_gap=g_direct)
        S_, G_ = N, N + 1
        nb = [list(zip(rm["adj"][i], rm["adj_w"][i])) for i in range(N)] + [[], []]
        for j, g, w in ends[0]:
            if not g < 0.0:
                nb[S_].append((j, w))
        for j, g, w in ends[1]:
            if not g < 0.0:
                nb[j].append((G_, w))
        if not g_direct < 0.0:
            nb[S_].append((G_, float(np.sqrt(dist2(qs, qg)))))
        dist = np.full(N + 2, np.inf)
        pred = np.full(N + 2, -1)
        done = np.zeros(N + 2, dtype=bool)
        dist[S_] = 0.0
        heap = [(0.0, S_)]
        while heap:
            dv, v = heapq.heappop(heap)
            if done[v]:
                continue
            done[v] = True
            if v == G_:
                break
            for w_, wt in nb[v]:
                cand = dv + wt
                if not done[w_] and cand < dist[w_]:
                    dist[w_] = cand
                    pred[w_] = v
                    heapq.heappush(heap, (cand, w_))
        if done[G_]:
            path = [G_]
            while path[-1] != S_:
                path.append(int(pred[path[-1]]))
            path = path[::-1]
            n_path = len(path) - 2
            allu = np.concatenate([nodes, qs[None], qg[None]])
            pts, s = allu[path], dist[path]
        else:
            path, n_path = [S_, G_], -1
            pts, s = np.stack([qs, qg]), np.array([0.0, np.sqrt(dist2(qs, qg))])
    Q = resample_linear(pts, s, H)
    seeds = np.repeat(Q[None], S, axis=0)
    if bumps is not None:
        bumps = np.asarray(bumps, dtype=np.float64).reshape(S, H + 1, 3 * n)
        umax = np.asarray(robot.u_max[:n], dtype=np.float64)
        for q in range(1, S):
            x = (Q + bumps[q]).reshape(H + 1, n, 3)
            peak = np.abs(x).max(axis=2)
            scale = np.minimum(1.0, umax[None, :] / np.maximum(peak, 1e-300))
            seeds[q] = (x * scale[:, :, None]).reshape(H + 1, 3 * n)
    out.update(path=path, n_path=n_path, seeds=seeds.reshape(S, H + 1, n, 3))
    return out
