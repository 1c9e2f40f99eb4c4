"""Python binding of libcrsolver.so (the gfx950 CR-Solver hot path).

Argument marshalling only: every entry point checks shapes, dtypes and devices of
torch tensors, then passes raw device pointers and the current HIP stream to the
C ABI declared in include/cr_solver.h.  There is no CPU fallback: if the HIP
library is missing the import of this module raises.

Layouts are structure-of-arrays with the batch index fastest (see cr_solver.h):
  u       [3n, B]          tendon displacements, row 3*i + j
  poses   [12, B]          3x4 row-major [R | p]
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrsolver.so")
MAX_SEG = 6

CR_OK, CR_EINVAL, CR_ENOMEM, CR_EDEVICE, CR_EUNSUPPORTED = 0, 1, 2, 3, 4
F32, F64 = 0, 1
KIND = {"ik": 0, "path": 1, "traj": 2}
SOLVED, LIMIT_VIOLATION, COLLISION, NONFINITE, NOT_CONVERGED = 1, 2, 4, 8, 16

EXPORTS = ("cr_fk", "cr_cost_grad", "cr_solve_ik", "cr_solve_ik_workspace", "cr_solve_ik_static", "cr_solve_path", "cr_solve_traj",
           "cr_solve_traj_workspace", "cr_solve_batch", "cr_solve_batch_workspace", "cr_baseline_solve_ik",
           "cr_baseline_solve_path", "cr_baseline_solve_traj", "cr_baseline_traj_workspace",
           "cr_select_top", "cr_sample_seeds", "cr_prm_build", "cr_prm_query", "cr_calib_valu",
           "cr_timing_enable", "cr_timing_read", "cr_ik_flop_tally", "cr_autotune_enable", "cr_autotune_clear", "cr_autotune_force",
           "cr_autotune_report", "cr_status_string", "cr_last_error")


class CRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class _Robot(C.Structure):
    _fields_ = [("n_seg", C.c_int32), ("pts_per_seg", C.c_int32),
                ("L", C.c_double * MAX_SEG), ("r", C.c_double * MAX_SEG),
                ("u_max", C.c_double * MAX_SEG), ("theta_max", C.c_double),
                ("extensible", C.c_int32), ("L_min", C.c_double * MAX_SEG), ("L_max", C.c_double * MAX_SEG),
                ("self_collision", C.c_int32)]


class _Spheres(C.Structure):
    _fields_ = [("n_sph", C.c_int32), ("per_problem", C.c_int32), ("sph", C.c_void_p), ("ld", C.c_int64),
                ("n_poly", C.c_int32), ("n_planes", C.c_int32), ("planes", C.c_void_p), ("plane_ld", C.c_int64)]


class _PrmOpts(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("k", C.c_int32), ("n_check", C.c_int32), ("max_attempts", C.c_int32),
                ("key0", C.c_uint64), ("key1", C.c_uint64)]


PRM_NONE = -(2 ** 31)


class _Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("robot", C.c_int32), ("H", C.c_int32), ("S", C.c_int32),
                ("n_sph", C.c_int32), ("pad", C.c_int32), ("task_off", C.c_int64), ("seed_off", C.c_int64),
                ("sph_off", C.c_int64), ("out_off", C.c_int64)]


class _Weights(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "w_pos", "w_rot", "rho_lim", "rho_curv", "rho_coll", "margin", "rho_eq",
        "w_len", "w_vel", "w_acc", "v_max", "a_max", "dt")]


class _Opts(C.Structure):
    _fields_ = [("n_final", C.c_int32), ("k_init", C.c_int32), ("k_final", C.c_int32),
                ("ls_max", C.c_int32), ("fp64_refine", C.c_int32), ("lambda0", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("dup_eps", C.c_double),
                ("k_seed", C.c_int32)]


@dataclass
class Robot:
    """Piecewise-constant-curvature robot with three tendons per segment (Sec. III)."""
    L: list
    r: list
    u_max: list
    pts_per_seg: int = 10
    theta_max: float = math.pi
    L_min: list = None   # extensible segments: length bounds (m); both given <=> the
    L_max: list = None   # common mode of each segment's tendons is its extension
    self_collision: bool = False   # contact between non-adjacent segments counts (eq. 10)

    @property
    def n(self) -> int:
        return len(self.L)

    @property
    def extensible(self) -> bool:
        return self.L_min is not None and self.L_max is not None

    @property
    def nc(self) -> int:
        """coordinates per segment in the solver (a, b and, if extensible, e)"""
        return 3 if self.extensible else 2

    def c(self) -> _Robot:
        s = _Robot()
        s.n_seg, s.pts_per_seg = self.n, self.pts_per_seg
        for i in range(self.n):
            s.L[i], s.r[i], s.u_max[i] = self.L[i], self.r[i], self.u_max[i]
        s.theta_max = self.theta_max
        if self.extensible:
            s.extensible = 1
            for i in range(self.n):
                s.L_min[i], s.L_max[i] = self.L_min[i], self.L_max[i]
        s.self_collision = 1 if self.self_collision else 0
        return s


@dataclass
class Weights:
    """Weights of the penalised cost, eq. (17)."""
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
    """Two-stage solver options (Algorithm 1) and LM damping."""
    n_final: int = 8
    k_init: int = 150
    k_final: int = 50
    ls_max: int = 4
    fp64_refine: int = 1
    lambda0: float = 1e-3
    lambda_min: float = 1e-12
    lambda_max: float = 1e12
    dup_eps: float = 1e-3
    k_seed: int = 0

    def c(self) -> _Opts:
        return _Opts(self.n_final, self.k_init, self.k_final, self.ls_max, self.fp64_refine,
                     self.lambda0, self.lambda_min, self.lambda_max, self.dup_eps, self.k_seed)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2607_11340_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    R, S, W, O = C.POINTER(_Robot), C.POINTER(_Spheres), C.POINTER(_Weights), C.POINTER(_Opts)
    L.cr_fk.argtypes = [R, i64, vp, i64, vp, vp, vp, C.c_int, vp]
    L.cr_cost_grad.argtypes = [i32, R, S, W, i64, i32, i32, vp, vp, vp, vp, vp, C.c_int, vp]
    L.cr_solve_ik.argtypes = [R, S, i64, vp, i32, vp, W, O, vp, vp, vp, vp, C.c_size_t, C.c_int, vp]
    L.cr_solve_ik_static.argtypes = [R, S, i64, vp, i32, vp, W, O, vp, vp, vp, C.c_int, vp]
    L.cr_solve_path.argtypes = [R, S, i64, i32, vp, i32, vp, W, O, vp, vp, vp, vp, C.c_size_t, C.c_int, vp]
    L.cr_solve_traj.argtypes = [R, S, i64, i32, vp, i32, vp, W, O, vp, vp, vp, vp, C.c_size_t, C.c_int, vp]
    L.cr_solve_traj_workspace.argtypes = [R, i64, i32, i32, O, C.c_int]
    L.cr_solve_traj_workspace.restype = C.c_size_t
    L.cr_baseline_solve_ik.argtypes = [R, S, i64, vp, i32, vp, W, O, vp, vp, vp, vp, C.c_size_t, vp]
    L.cr_baseline_solve_path.argtypes = [R, S, i64, i32, vp, i32, vp, W, O, vp, vp, vp, vp, C.c_size_t, vp]
    L.cr_baseline_solve_traj.argtypes = [R, S, i64, i32, vp, i32, vp, W, O, vp, vp, vp, vp, C.c_size_t, vp]
    L.cr_baseline_traj_workspace.argtypes = [R, i32, i32, O]
    L.cr_baseline_traj_workspace.restype = C.c_size_t
    PR = C.POINTER(_Problem)
    L.cr_solve_batch.argtypes = [R, i32, PR, i64, vp, vp, vp, W, O, vp, vp, vp, vp, C.c_size_t, C.c_int, i32, vp]
    L.cr_solve_batch_workspace.argtypes = [R, i32, PR, i64, O, C.c_int]
    L.cr_solve_batch_workspace.restype = C.c_size_t
    L.cr_solve_ik_workspace.argtypes = [R, i64, i32, O, C.c_int]
    L.cr_solve_ik_workspace.restype = C.c_size_t
    L.cr_select_top.argtypes = [i64, i32, i32, vp, vp, vp, vp, i32, C.c_double, vp, C.c_int, vp]
    L.cr_calib_valu.argtypes = [i32, i64, i32, vp, vp]
    L.cr_timing_enable.argtypes = [i32]
    L.cr_timing_enable.restype = None
    L.cr_timing_read.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.cr_ik_flop_tally.argtypes = [R, W, O, i64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]
    L.cr_autotune_enable.argtypes = [i32]
    L.cr_autotune_enable.restype = None
    L.cr_autotune_force.argtypes = [i32]
    L.cr_autotune_force.restype = None
    L.cr_autotune_clear.argtypes = []
    L.cr_autotune_clear.restype = None
    L.cr_autotune_report.argtypes = [C.c_char_p, i64]
    L.cr_autotune_report.restype = i64
    L.cr_sample_seeds.argtypes = [R, S, i64, i32, C.c_uint64, C.c_uint64, i32, vp, vp, vp]
    PO = C.POINTER(_PrmOpts)
    L.cr_prm_build.argtypes = [R, S, i64, PO, vp, vp, vp, vp, vp, vp, vp]
    L.cr_prm_query.argtypes = [R, S, i64, PO, vp, vp, vp, vp, vp, vp, i32, i32, vp, i32, vp, vp, vp, vp]
    L.cr_status_string.argtypes = [C.c_int]
    L.cr_status_string.restype = C.c_char_p
    L.cr_last_error.restype = C.c_char_p
    for name in ("cr_fk", "cr_cost_grad", "cr_solve_ik", "cr_solve_ik_static", "cr_solve_path", "cr_solve_traj", "cr_solve_batch",
                 "cr_baseline_solve_ik", "cr_baseline_solve_path", "cr_baseline_solve_traj", "cr_select_top",
                 "cr_sample_seeds", "cr_prm_build", "cr_prm_query", "cr_timing_read", "cr_ik_flop_tally", "cr_calib_valu"):
        getattr(L, name).restype = C.c_int
    return L


lib = _load()


def _check(rc: int):
    if rc != CR_OK:
        raise CRError(rc, lib.cr_last_error().decode())


def _stream(t: torch.Tensor):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dt(dtype) -> int:
    if dtype in (torch.float32, "f32", F32):
        return F32
    if dtype in (torch.float64, "f64", F64):
        return F64
    raise ValueError(f"dtype {dtype} not supported")


def _tdt(code: int):
    return torch.float64 if code == F64 else torch.float32


def _need(t, shape, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _spheres_c(spheres, dtype, polytopes=None) -> _Spheres:
    """spheres: None, or (tensor [4, M] shared) or (tensor [4, M*P], per_problem=True).
    polytopes (convex obstacles, IK only): None, or (tensor [4, ld], per_problem,
    n_poly, n_planes): plane f of polytope j at column j*n_planes + f (+ p*n_poly*
    n_planes per problem), rows nx, ny, nz, d of the half-space n.x <= d."""
    out = _Spheres(0, 0, None, 0, 0, 0, None, 0)
    pp = None
    if spheres is not None:
        t, per_problem, M = spheres
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.shape[0] != 4:
            raise ValueError("spheres must be a contiguous CUDA tensor [4, ld] of the call's dtype")
        out.n_sph, out.sph, out.ld = int(M), C.c_void_p(t.data_ptr()), int(t.shape[1])
        pp = bool(per_problem)
    if polytopes is not None:
        t, per_problem, n_poly, n_planes = polytopes
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.shape[0] != 4:
            raise ValueError("polytopes must be a contiguous CUDA tensor [4, ld] of the call's dtype")
        if pp is not None and pp != bool(per_problem):
            raise ValueError("spheres and polytopes must agree on per_problem")
        out.n_poly, out.n_planes = int(n_poly), int(n_planes)
        out.planes, out.plane_ld = C.c_void_p(t.data_ptr()), int(t.shape[1])
        pp = bool(per_problem)
    out.per_problem = 1 if pp else 0
    return out


def fk(robot: Robot, u: torch.Tensor, arc=True, frames=True, points=False):
    """Forward kinematics of B configurations u [3n, B]; returns a dict of
    arc [3n, B], frames [12n, B], pts [3nK, B] (those requested)."""
    dt = _dt(u.dtype)
    n, B = robot.n, u.shape[1]
    _need(u, (3 * n, B), u.dtype, "u")
    out = {}
    a = torch.empty((3 * n, B), dtype=u.dtype, device=u.device) if arc else None
    f = torch.empty((12 * n, B), dtype=u.dtype, device=u.device) if frames else None
    p = torch.empty((3 * n * robot.pts_per_seg, B), dtype=u.dtype, device=u.device) if points else None
    rc = robot.c()
    _check(lib.cr_fk(C.byref(rc), B, _ptr(u), B, _ptr(a), _ptr(f), _ptr(p), dt, _stream(u)))
    if arc:
        out["arc"] = a
    if frames:
        out["frames"] = f
    if points:
        out["pts"] = p
    return out


def ik_workspace_bytes(robot: Robot, P: int, S: int, opts: Opts, dtype) -> int:
    rc, oc = robot.c(), opts.c()
    return int(lib.cr_solve_ik_workspace(C.byref(rc), P, S, C.byref(oc), _dt(dtype)))


def sample_seeds(robot: Robot, P: int, S: int, key=(0, 0), max_attempts: int = 8, spheres=None,
                 device="cuda"):
    """SampleSeeds of Algorithm 1 on the device (cr_sample_seeds): S seeds for each
    of P problems inside the bounds, colliding ones drawn again up to max_attempts
    times.  key: two 64-bit integers; spheres as for solve_ik (float64).  Returns
    (u_seed [3n, S*P] float64, column p*S + s; attempts [S*P] int32, negative for
    a seed that still collides)."""
    u = torch.empty((3 * robot.n, S * P), dtype=torch.float64, device=device)
    att = torch.empty((S * P,), dtype=torch.int32, device=device)
    sp = _spheres_c(spheres, torch.float64)
    rc = robot.c()
    _check(lib.cr_sample_seeds(C.byref(rc), C.byref(sp), P, S,
                               int(key[0]) & (2 ** 64 - 1), int(key[1]) & (2 ** 64 - 1), max_attempts, _ptr(u),
                               _ptr(att), _stream(u)))
    return u, att


@dataclass
class PrmOpts:
    """Roadmap and query parameters of the PRM exploration stage (Algorithm 2)."""
    n_nodes: int = 1024
    k: int = 10
    n_check: int = 8
    max_attempts: int = 8
    key: tuple = (0, 0)

    def c(self) -> _PrmOpts:
        return _PrmOpts(self.n_nodes, self.k, self.n_check, self.max_attempts, int(self.key[0]) & (2 ** 64 - 1),
                        int(self.key[1]) & (2 ** 64 - 1))


def prm_build(robot: Robot, P: int, prm: PrmOpts, spheres=None, device="cuda"):
    """Offline roadmaps of P scenes (cr_prm_build).  spheres as for solve_traj
    (float64).  Returns a dict of device tensors: nodes [3n, N*P] float64,
    attempts [N*P], nbr [k, N*P], adj_off [(N+1)*P], adj [2kN*P] int32 and
    adj_w [2kN*P] float64."""
    n, N, k = robot.n, prm.n_nodes, prm.k
    B = N * P
    out = dict(nodes=torch.empty((3 * n, B), dtype=torch.float64, device=device),
               attempts=torch.empty((B,), dtype=torch.int32, device=device),
               nbr=torch.empty((k, B), dtype=torch.int32, device=device),
               adj_off=torch.empty(((N + 1) * P,), dtype=torch.int32, device=device),
               adj=torch.empty((2 * k * B,), dtype=torch.int32, device=device),
               adj_w=torch.empty((2 * k * B,), dtype=torch.float64, device=device))
    rc, pc = robot.c(), prm.c()
    sp = _spheres_c(spheres, torch.float64)
    t = out["nodes"]
    _check(lib.cr_prm_build(C.byref(rc), C.byref(sp), P, C.byref(pc), _ptr(t), _ptr(out["attempts"]),
                            _ptr(out["nbr"]), _ptr(out["adj_off"]), _ptr(out["adj"]), _ptr(out["adj_w"]), _stream(t)))
    return out


def prm_query(robot: Robot, prm: PrmOpts, u_start_goal: torch.Tensor, H: int, S: int, roadmap: dict = None,
              bump: torch.Tensor = None, linear: bool = False, spheres=None, out=None, path: bool = False):
    """Online queries (cr_prm_query): u_start_goal [6n, P] float64 on the roadmaps
    of prm_build (None with linear=True).  bump: None or [3n, (H+1)*S*P] float64.
    Returns (u_seed [3n, (H+1)*S*P] float64, n_path [P] int32, path [N+2, P] int32
    or None)."""
    n = robot.n
    P = u_start_goal.shape[1]
    _need(u_start_goal, (6 * n, P), torch.float64, "u_start_goal")
    cols = (H + 1) * S * P
    if bump is not None:
        _need(bump, (3 * n, cols), torch.float64, "bump")
    dev = u_start_goal.device
    if out is None:
        out = (torch.empty((3 * n, cols), dtype=torch.float64, device=dev),
               torch.empty((P,), dtype=torch.int32, device=dev))
    useed, npath = out
    pth = torch.empty((prm.n_nodes + 2, P), dtype=torch.int32, device=dev) if path else None
    rm = roadmap or {}
    if not linear:
        N, k = prm.n_nodes, prm.k
        _need(rm["nodes"], (3 * n, N * P), torch.float64, "nodes")
        _need(rm["adj"], (2 * k * N * P,), torch.int32, "adj")
    rc, pc = robot.c(), prm.c()
    sp = _spheres_c(spheres, torch.float64)
    _check(lib.cr_prm_query(C.byref(rc), C.byref(sp), P, C.byref(pc), _ptr(rm.get("nodes")), _ptr(rm.get("attempts")),
                            _ptr(rm.get("adj_off")), _ptr(rm.get("adj")), _ptr(rm.get("adj_w")), _ptr(u_start_goal),
                            H, S, _ptr(bump), 1 if linear else 0, _ptr(useed), _ptr(npath), _ptr(pth),
                            _stream(u_start_goal)))
    return useed, npath, pth


def solve_ik(robot: Robot, T_target: torch.Tensor, u_seed: torch.Tensor, weights: Weights = None,
             opts: Opts = None, dtype=torch.float32, spheres=None, workspace: torch.Tensor = None, out=None,
             polytopes=None):
    """Two-stage IK (Algorithm 1).  T_target [12, P] float64, u_seed [3n, S*P] float64
    (column p*S + s).  `dtype` is the stage-1 precision.  Returns (u [3n, P],
    err [2, P] (position m, rotation rad), status [P] int32)."""
    weights = weights or Weights()
    opts = opts or Opts()
    n = robot.n
    P = T_target.shape[1]
    S = u_seed.shape[1] // max(P, 1)
    _need(T_target, (12, P), torch.float64, "T_target")
    _need(u_seed, (3 * n, S * P), torch.float64, "u_seed")
    dev = T_target.device
    if out is None:
        out = (torch.empty((3 * n, P), dtype=torch.float64, device=dev),
               torch.empty((2, P), dtype=torch.float64, device=dev),
               torch.empty((P,), dtype=torch.int32, device=dev))
    u_out, err, st = out
    rc, wc, oc = robot.c(), weights.c(), opts.c()
    sc = _spheres_c(spheres, torch.float64, polytopes)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
    _check(lib.cr_solve_ik(C.byref(rc), C.byref(sc), P, _ptr(T_target), S, _ptr(u_seed), C.byref(wc),
                           C.byref(oc), _ptr(u_out), _ptr(err), _ptr(st), ws_ptr, ws_bytes, _dt(dtype),
                           _stream(T_target)))
    return u_out, err, st


STATIC_SCRATCH_BYTES = 64 << 20


def solve_ik_static(robot: Robot, T_target: torch.Tensor, u_seed: torch.Tensor, weights: Weights = None,
                    opts: Opts = None, dtype=torch.float32, spheres=None, out=None, polytopes=None):
    """solve_ik through cr_solve_ik_static: no workspace and no device allocation
    inside the call (its scratch is the library's static per-GPU buffer).  `out`
    (u, err, status) must be given by callers that cannot allocate; when None,
    this wrapper allocates the outputs before the call."""
    weights = weights or Weights()
    opts = opts or Opts()
    n = robot.n
    P = T_target.shape[1]
    S = u_seed.shape[1] // max(P, 1)
    _need(T_target, (12, P), torch.float64, "T_target")
    _need(u_seed, (3 * n, S * P), torch.float64, "u_seed")
    dev = T_target.device
    if out is None:
        out = (torch.empty((3 * n, P), dtype=torch.float64, device=dev),
               torch.empty((2, P), dtype=torch.float64, device=dev),
               torch.empty((P,), dtype=torch.int32, device=dev))
    u_out, err, st = out
    rc, wc, oc = robot.c(), weights.c(), opts.c()
    sc = _spheres_c(spheres, torch.float64, polytopes)
    _check(lib.cr_solve_ik_static(C.byref(rc), C.byref(sc), P, _ptr(T_target), S, _ptr(u_seed), C.byref(wc),
                                  C.byref(oc), _ptr(u_out), _ptr(err), _ptr(st), _dt(dtype), _stream(T_target)))
    return u_out, err, st


def baseline_solve_ik(robot: Robot, T_target: torch.Tensor, u_seed: torch.Tensor, weights: Weights = None,
                      opts: Opts = None, out=None, spheres=None):
    """The plain per-problem FP32 comparison solve (cr_baseline_solve_ik); arrays
    and spheres as solve_ik."""
    weights = weights or Weights()
    opts = opts or Opts()
    n, P = robot.n, T_target.shape[1]
    S = u_seed.shape[1] // max(P, 1)
    _need(T_target, (12, P), torch.float64, "T_target")
    _need(u_seed, (3 * n, S * P), torch.float64, "u_seed")
    dev = T_target.device
    if out is None:
        out = (torch.empty((3 * n, P), dtype=torch.float64, device=dev),
               torch.empty((2, P), dtype=torch.float64, device=dev),
               torch.empty((P,), dtype=torch.int32, device=dev))
    u_out, err, st = out
    rc, wc, oc = robot.c(), weights.c(), opts.c()
    sc = _spheres_c(spheres, torch.float64)
    _check(lib.cr_baseline_solve_ik(C.byref(rc), C.byref(sc), P, _ptr(T_target), S, _ptr(u_seed), C.byref(wc),
                                    C.byref(oc), _ptr(u_out), _ptr(err), _ptr(st), None, 0, _stream(T_target)))
    return u_out, err, st


def traj_workspace_bytes(robot: Robot, P: int, H: int, S: int, opts: Opts, dtype) -> int:
    rc, oc = robot.c(), opts.c()
    return int(lib.cr_solve_traj_workspace(C.byref(rc), P, H, S, C.byref(oc), _dt(dtype)))


def _solve_traj(kind: str, robot: Robot, task: torch.Tensor, u_seed: torch.Tensor, H: int, weights, opts, dtype,
                spheres, workspace, out, baseline=False):
    weights = weights or Weights()
    opts = opts or Opts(n_final=4, k_init=100, k_final=20)
    n, T = robot.n, H + 1
    P = task.shape[1] // (T if kind == "path" else 1)
    S = max(u_seed.shape[1] // max(T * P, 1), 1)
    if kind == "path":
        _need(task, (12, T * P), torch.float64, "T_ref")
    else:
        _need(task, (6 * n, P), torch.float64, "u_start_goal")
    _need(u_seed, (3 * n, T * S * P), torch.float64, "u_seed")
    dev = task.device
    if out is None:
        out = (torch.empty((3 * n, T * P), dtype=torch.float64, device=dev),
               torch.empty((2, P), dtype=torch.float64, device=dev),
               torch.empty((P,), dtype=torch.int32, device=dev))
    u_out, err, st = out
    rc, wc, oc = robot.c(), weights.c(), opts.c()
    sc = _spheres_c(spheres, torch.float64)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
    if baseline:
        fn = lib.cr_baseline_solve_path if kind == "path" else lib.cr_baseline_solve_traj
        _check(fn(C.byref(rc), C.byref(sc), P, H, _ptr(task), S, _ptr(u_seed), C.byref(wc), C.byref(oc),
                  _ptr(u_out), _ptr(err), _ptr(st), ws_ptr, ws_bytes, _stream(task)))
        return u_out, err, st
    fn = lib.cr_solve_path if kind == "path" else lib.cr_solve_traj
    _check(fn(C.byref(rc), C.byref(sc), P, H, _ptr(task), S, _ptr(u_seed), C.byref(wc), C.byref(oc), _ptr(u_out),
              _ptr(err), _ptr(st), ws_ptr, ws_bytes, _dt(dtype), _stream(task)))
    return u_out, err, st


def solve_path(robot: Robot, T_ref: torch.Tensor, u_seed: torch.Tensor, H: int, weights: Weights = None,
               opts: Opts = None, dtype=torch.float32, spheres=None, workspace=None, out=None):
    """Two-stage path following (eq. 16).  T_ref [12, (H+1)*P] float64 (column p*(H+1)+t),
    u_seed [3n, (H+1)*S*P] float64 (column (p*S+s)*(H+1)+t).  Returns (u [3n, (H+1)*P],
    err [2, P] (largest position m / rotation rad error over waypoints), status [P])."""
    return _solve_traj("path", robot, T_ref, u_seed, H, weights, opts, dtype, spheres, workspace, out)


def solve_traj(robot: Robot, u_start_goal: torch.Tensor, u_seed: torch.Tensor, H: int, weights: Weights = None,
               opts: Opts = None, dtype=torch.float32, spheres=None, workspace=None, out=None):
    """Two-stage trajectory planning (eq. 11-15).  u_start_goal [6n, P] float64 (start then
    goal tendon displacements), u_seed as in solve_path.  err: largest endpoint error."""
    return _solve_traj("traj", robot, u_start_goal, u_seed, H, weights, opts, dtype, spheres, workspace, out)


def baseline_solve_path(robot: Robot, T_ref: torch.Tensor, u_seed: torch.Tensor, H: int, weights: Weights = None,
                        opts: Opts = None, spheres=None, out=None):
    """The plain per-problem FP32 comparison solve for path following
    (cr_baseline_solve_path); arrays as solve_path."""
    return _solve_traj("path", robot, T_ref, u_seed, H, weights, opts, torch.float32, spheres, None, out,
                       baseline=True)


def baseline_solve_traj(robot: Robot, u_start_goal: torch.Tensor, u_seed: torch.Tensor, H: int,
                        weights: Weights = None, opts: Opts = None, spheres=None, out=None):
    """The plain per-problem FP32 comparison solve for trajectories
    (cr_baseline_solve_traj); arrays as solve_traj."""
    return _solve_traj("traj", robot, u_start_goal, u_seed, H, weights, opts, torch.float32, spheres, None, out,
                       baseline=True)


BATCH_GRAPH = 1
BATCH_PERSISTENT = 2


class Batch:
    """An uneven batch packed in the layout cr_solve_batch reads.  Each problem is
    a dict: kind ('ik'|'path'|'traj'), robot (index), H, task (IK [3,4] pose;
    PATH [H+1,3,4] poses; TRAJ (u_start [n,3], u_goal [n,3])), seeds
    [S, H+1, n, 3] (IK: [S, n, 3]) and optionally spheres [M, 4]."""

    def __init__(self, robots, problems):
        import numpy as np
        self.robots = list(robots)
        P = len(problems)
        self.table = (_Problem * max(P, 1))()
        task, seed, sph = [], [], []
        off = dict(task=0, seed=0, sph=0, out=0)
        self.out_shape = []
        for i, pb in enumerate(problems):
            n = self.robots[pb["robot"]].n
            kind = KIND[pb["kind"]]
            H = int(pb.get("H", 0))
            Tn = H + 1
            if pb["kind"] == "ik":
                t = np.asarray(pb["task"], dtype=np.float64).reshape(12)
            elif pb["kind"] == "path":
                t = np.asarray(pb["task"], dtype=np.float64).reshape(Tn, 12).T.reshape(-1)      # [12][Tn]
            else:
                us, ug = pb["task"]
                t = np.concatenate([np.ravel(us), np.ravel(ug)]).astype(np.float64)
            s = np.asarray(pb["seeds"], dtype=np.float64).reshape(-1, Tn, n * 3)             # [S, Tn, 3n]
            S = s.shape[0]
            s = s.reshape(S * Tn, 3 * n).T.reshape(-1)                                        # [3n][S*Tn]
            m = np.zeros((0, 4)) if pb.get("spheres") is None else np.asarray(pb["spheres"], dtype=np.float64)
            r = self.table[i]
            r.kind, r.robot, r.H, r.S, r.n_sph, r.pad = kind, pb["robot"], H, S, len(m), 0
            r.task_off, r.seed_off, r.sph_off, r.out_off = off["task"], off["seed"], off["sph"], off["out"]
            task.append(t)
            seed.append(s)
            sph.append(m.T.reshape(-1))
            off["task"] += t.size
            off["seed"] += s.size
            off["sph"] += m.size
            off["out"] += 3 * n * Tn
            self.out_shape.append((r.out_off, n, Tn, kind))
        self.P = P
        cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0)
        self.task = cat(task)
        self.seed = cat(seed)
        self.sph = cat(sph)
        self.n_out = off["out"]

    def unpack(self, u_flat):
        """Per-problem outputs [H+1, n, 3] (IK: [n, 3]) from the packed u_out."""
        res = []
        for (o, n, Tn, kind) in self.out_shape:
            u = u_flat[o:o + 3 * n * Tn].reshape(3 * n, Tn).T.reshape(Tn, n, 3)
            res.append(u[0] if kind == 0 else u)
        return res


def batch_workspace_bytes(batch: "Batch", opts, dtype) -> int:
    rob = (_Robot * len(batch.robots))(*[r.c() for r in batch.robots])
    oc = (_Opts * 3)(*[o.c() for o in opts])
    return int(lib.cr_solve_batch_workspace(rob, len(batch.robots), batch.table, batch.P, oc, _dt(dtype)))


def solve_batch(batch: "Batch", weights, opts, dtype=torch.float32, device="cuda", graph=False, workspace=None,
                dev_arrays=None, out=None, persistent=False):
    """cr_solve_batch on a packed Batch.  weights, opts: 3 each, indexed by kind
    (ik, path, traj).  persistent: IK stage 1 as one work-queue kernel per group
    with SelectTop fused in.  Returns (u_out flat [device], err [2, P], status [P])."""
    if dev_arrays is None:
        mk = lambda a: torch.tensor(a if a.size else [0.0], dtype=torch.float64, device=device)
        dev_arrays = (mk(batch.task), mk(batch.seed), mk(batch.sph))
    task, seed, sph = dev_arrays
    if out is None:
        out = (torch.empty(max(batch.n_out, 1), dtype=torch.float64, device=device),
               torch.empty((2, max(batch.P, 1)), dtype=torch.float64, device=device),
               torch.empty(max(batch.P, 1), dtype=torch.int32, device=device))
    u, err, st = out
    rob = (_Robot * len(batch.robots))(*[r.c() for r in batch.robots])
    wc = (_Weights * 3)(*[w.c() for w in weights])
    oc = (_Opts * 3)(*[o.c() for o in opts])
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
    _check(lib.cr_solve_batch(rob, len(batch.robots), batch.table, batch.P, _ptr(task), _ptr(seed), _ptr(sph), wc, oc,
                              _ptr(u), _ptr(err), _ptr(st), ws_ptr, ws_bytes, _dt(dtype),
                              (BATCH_GRAPH if graph else 0) | (BATCH_PERSISTENT if persistent else 0),
                              _stream(task)))
    return u, err, st


def select_top(z: torch.Tensor, e: torch.Tensor, pen: torch.Tensor, failed, P: int, S: int, n_final: int,
               dup_eps: float = 1e-3):
    """SelectTop of Algorithm 1 per problem.  z [nz, S*P], e/pen [S*P], failed int32 [S*P]
    or None.  Returns idx [n_final, P] int32 (seed index within its problem, -1 = empty)."""
    dt = _dt(e.dtype)
    nz = z.shape[0]
    _need(z, (nz, S * P), e.dtype, "z")
    _need(e, (S * P,), e.dtype, "e")
    _need(pen, (S * P,), e.dtype, "pen")
    if failed is not None:
        _need(failed, (S * P,), torch.int32, "failed")
    idx = torch.empty((n_final, P), dtype=torch.int32, device=e.device)
    _check(lib.cr_select_top(P, S, nz, _ptr(z), _ptr(e), _ptr(pen), _ptr(failed), n_final, dup_eps,
                             _ptr(idx), dt, _stream(e)))
    return idx


@dataclass
class CostProblem:
    """A batch of P problems x S seeds x (H+1) waypoints for cr_cost_grad.
    task: IK [12, P] poses; PATH [12, (H+1)*P] reference poses (column p*(H+1)+t);
    TRAJ [6n, P] (u_start then u_goal).  spheres: None or (tensor [4, ld], per_problem, M).
    polytopes (IK only): None or (tensor [4, ld], per_problem, n_poly, n_planes)."""
    robot: Robot
    kind: str
    P: int
    S: int
    H: int
    task: torch.Tensor
    weights: Weights = field(default_factory=Weights)
    spheres: tuple = None
    polytopes: tuple = None


def cost_grad(pb: CostProblem, u: torch.Tensor, grad: bool = True, grad_scale: torch.Tensor = None):
    """Penalised cost (eq. 17) per seed [S*P] and, if grad, dC/du like u [3n, (H+1)*S*P]."""
    dt = _dt(u.dtype)
    n, T = pb.robot.n, pb.H + 1
    B = pb.P * pb.S * T
    _need(u, (3 * n, B), u.dtype, "u")
    if pb.task.dtype != u.dtype:
        raise ValueError("task must have the dtype of u")
    cost = torch.empty((pb.S * pb.P,), dtype=u.dtype, device=u.device)
    g = torch.empty_like(u) if grad else None
    if grad_scale is not None:
        _need(grad_scale, (pb.S * pb.P,), u.dtype, "grad_scale")
    rc, wc = pb.robot.c(), pb.weights.c()
    sc = _spheres_c(pb.spheres, u.dtype, pb.polytopes)
    _check(lib.cr_cost_grad(KIND[pb.kind], C.byref(rc), C.byref(sc), C.byref(wc), pb.P, pb.H, pb.S,
                            _ptr(pb.task), _ptr(u), _ptr(cost), _ptr(g), _ptr(grad_scale), dt, _stream(u)))
    return (cost, g) if grad else cost


class CostGrad(torch.autograd.Function):
    """cost = CostGrad.apply(u, problem): forward evaluates the cost only; backward
    recomputes the transforms and runs the adjoint kernel, scaled per seed by the
    upstream gradient inside the kernel.  Only u is saved."""

    @staticmethod
    def forward(ctx, u, problem):
        ctx.problem = problem
        ctx.save_for_backward(u)
        return cost_grad(problem, u.detach(), grad=False)

    @staticmethod
    def backward(ctx, gcost):
        (u,) = ctx.saved_tensors
        _, g = cost_grad(ctx.problem, u.detach(), grad=True, grad_scale=gcost.contiguous())
        return g, None


def calib_valu(kind: int, blocks: int, iters: int, out: torch.Tensor):
    """One launch of the vector-ALU calibration loop `kind` (cr_calib_valu);
    out: float32 CUDA tensor of blocks * 256 elements."""
    _need(out, (blocks * 256,), torch.float32, "out")
    _check(lib.cr_calib_valu(int(kind), int(blocks), int(iters), _ptr(out), _stream(out)))


def autotune(on: bool = True):
    """Switch the library's launch autotuning on or off (cr_autotune_enable)."""
    lib.cr_autotune_enable(1 if on else 0)


def autotune_force(variant: int):
    """Run the given launch variant of every tunable kernel; -1 returns to normal
    operation (cr_autotune_force)."""
    lib.cr_autotune_force(int(variant))


def autotune_clear():
    """Forget every cached autotuning choice (cr_autotune_clear)."""
    lib.cr_autotune_clear()


def autotune_report() -> list:
    """The cached autotuning choices, one text line per key (cr_autotune_report)."""
    n = lib.cr_autotune_report(None, 0)
    buf = C.create_string_buffer(int(n) + 1)
    lib.cr_autotune_report(buf, n + 1)
    return [l for l in buf.value.decode().split("\n") if l]
