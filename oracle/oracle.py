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
