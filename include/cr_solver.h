/*
 * cr_solver.h -- C ABI of the MI355X (gfx950) CR-Solver hot path.
 *
 * CR-Solver (arXiv 2607.11340) solves inverse kinematics, path following and
 * trajectory planning of tendon-driven continuum robots as one penalised
 * nonlinear least-squares problem (Sec. IV-A, eq. 17), optimised from many seeds
 * at once by batched Levenberg-Marquardt (Sec. IV-C) inside a two-stage
 * exploration/refinement template (Sec. IV-B, Algorithm 1).
 *
 * General rules for every entry point:
 *  - No exception crosses this boundary; every call returns a cr_status.
 *  - Arrays marked [device] are device pointers (HIP global memory), arrays
 *    marked [host] are host pointers.  The caller owns all of them; the library
 *    never frees caller memory and keeps no pointer after the call returns.
 *  - Batched arrays are structure-of-arrays with the batch index fastest:
 *    element (component c, item b) lives at x[c * ld + b].  Unless an explicit
 *    `ld` is taken, ld equals the batch size of that array.
 *  - A pose is 12 components, the 3x4 row-major matrix [R | p]:
 *    c = 4*row + col, col 3 being the position (metres).
 *  - Tendon displacements u (metres) are 3 components per segment,
 *    c = 3*i + j for tendon j (at angle 2*pi*j/3 about the backbone) of
 *    segment i; u is the tendon length minus the segment length, eq. (4).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = default stream) and is
 *    stream-ordered; no call synchronises the host unless stated.
 *  - Shape, pointer, option and dtype errors return CR_EINVAL and launch
 *    nothing; HIP failures return CR_EDEVICE; cr_last_error() gives the text.
 *    Data-dependent trouble (NaN inputs, unreachable targets) never fails a
 *    call: it is reported per problem in the status bits below.
 */
#ifndef CR_SOLVER_H
#define CR_SOLVER_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CR_OK = 0,
  CR_EINVAL = 1,        /* invalid argument; nothing was launched */
  CR_ENOMEM = 2,        /* workspace too small or allocation failed */
  CR_EDEVICE = 3,       /* a HIP call failed */
  CR_EUNSUPPORTED = 4   /* valid request the library does not implement */
} cr_status;

/* Floating-point type of a call's arrays and arithmetic. */
typedef enum { CR_F32 = 0, CR_F64 = 1 } cr_dtype;

/* Task kinds of Sec. IV-A. */
typedef enum {
  CR_KIND_IK = 0,    /* inverse kinematics, eq. (8)-(10) */
  CR_KIND_PATH = 1,  /* path following, eq. (16) with the trajectory constraints */
  CR_KIND_TRAJ = 2   /* trajectory planning, eq. (11)-(15) */
} cr_kind;

/* Per-problem status bits written by the solve calls (success criterion of
 * Sec. V-B with the 1 mm / 1 degree thresholds). */
enum {
  CR_SOLVED = 1,          /* every check below passed */
  CR_LIMIT_VIOLATION = 2, /* a tendon exceeds its bound by > 1e-6 m or theta > theta_max */
  CR_COLLISION = 4,       /* a backbone point is inside an inflated sphere */
  CR_NONFINITE = 8,       /* every candidate had a non-finite cost */
  CR_NOT_CONVERGED = 16   /* position error > 1 mm or rotation error > 1 degree */
};

#define CR_MAX_SEG 6

/* Robot geometry (Sec. III, piecewise constant curvature, 3 tendons per segment). [host] */
typedef struct {
  int32_t n_seg;              /* number of segments n, 1..CR_MAX_SEG */
  int32_t pts_per_seg;        /* K backbone points per segment for collision, >= 1 */
  double L[CR_MAX_SEG];       /* segment arc length (m), > 0 */
  double r[CR_MAX_SEG];       /* tendon routing radius r_c (m), > 0; also the body radius */
  double u_max[CR_MAX_SEG];   /* bound on |u| of each tendon of the segment (m), > 0 */
  double theta_max;           /* bound on each bending angle (rad), default pi */
  int32_t extensible;         /* 0: inextensible segments, the common mode of each segment's
                                 three tendons is ignored (eq. 4 with L fixed).  1: extensible
                                 segments (the extendable robots of Sec. V-B): the common mode
                                 mean_j u_ij is the change of the segment's length,
                                 L_i = L[i] + mean_j u_ij, bounded by [L_min, L_max] (eq. 9);
                                 u_max then bounds the bending part u_ij - mean_j u_ij.
                                 Supported by cr_fk, cr_cost_grad (IK) and cr_solve_ik. */
  double L_min[CR_MAX_SEG];   /* extensible: segment length bounds (m), 0 < L_min <= L <= L_max */
  double L_max[CR_MAX_SEG];
  int32_t self_collision;     /* 1: contact between the robot's own non-adjacent segments
                                 (|i - j| >= 2) counts as collision (eq. 10): backbone points
                                 keep r_i + r_j apart, with the clearance penalty and margin
                                 of the obstacles; the status gets CR_COLLISION.  Supported by
                                 cr_cost_grad (IK) and cr_solve_ik (n_seg >= 3; fewer segments
                                 have no such pair). */
} cr_robot;

/* Obstacles.  [host] struct; the arrays are [device], in the call's dtype for
 * cr_cost_grad and double for the solve calls.
 * Spheres: sph[c * ld + m], c = cx, cy, cz, radius.
 * Convex polytopes (the convex pieces of Sec. V's obstacle model, in half-space
 * form; IK only: cr_cost_grad with kind IK, cr_solve_ik, cr_solve_ik_static):
 *   polytope j is the intersection of n_planes half-spaces n . x <= d; plane f of
 *   polytope j has components c = nx, ny, nz, d at planes[c * plane_ld + j *
 *   n_planes + f] (unit normals; an unused plane is n = 0 with a large d).  A
 *   backbone point x of segment i clears it when sd(x) - r_i >= 0 with the signed
 *   distance sd(x) = max_f (n_f . x - d_f) (exact inside and in the region of each
 *   face outside; below the distance near edges and corners outside); the
 *   clearance hinge of eq. (10) uses margin - (sd(x) - r_i).  Not supported with
 *   extensible segments or self contact (CR_EINVAL).
 * per_problem = 0: one set of obstacles shared by all problems;
 * per_problem = 1: problem p owns spheres m = p * n_sph .. p * n_sph + n_sph - 1
 *   and polytopes p * n_poly .. p * n_poly + n_poly - 1.
 * Zero-initialise the struct: n_sph = n_poly = 0 means no obstacles. */
typedef struct {
  int32_t n_sph;
  int32_t per_problem;
  const void* sph;
  int64_t ld;
  int32_t n_poly;      /* polytopes per problem (or shared), 0..256 */
  int32_t n_planes;    /* planes per polytope, 1..32 */
  const void* planes;
  int64_t plane_ld;
} cr_obstacles;
typedef cr_obstacles cr_spheres;

/* Weights of the penalised cost, eq. (17).  [host] */
typedef struct {
  double w_pos, w_rot;   /* pose residual weights (1/m, 1/rad) */
  double rho_lim;        /* tendon bound (and tendon velocity/acceleration bound) penalty */
  double rho_curv;       /* bending-angle bound penalty */
  double rho_coll;       /* obstacle clearance penalty */
  double margin;         /* safety margin delta of eq. (10) (m) */
  double rho_eq;         /* trajectory endpoint equality penalty */
  double w_len;          /* trajectory tip path-length weight, eq. (11) squared */
  double w_vel, w_acc;   /* quadratic tendon velocity / acceleration smoothness */
  double v_max, a_max;   /* tendon velocity / acceleration bounds, INFINITY = off */
  double dt;             /* time step of the finite differences */
} cr_weights;

/* Options of the two-stage solver (Algorithm 1) and of Levenberg-Marquardt.  [host] */
typedef struct {
  int32_t n_final;       /* N_final kept by SelectTop; 0 = plain method (no stage 2) */
  int32_t k_init;        /* stage-1 iterations */
  int32_t k_final;       /* stage-2 iterations */
  int32_t ls_max;        /* line-search trials, step 1, 1/2, 1/4, ... (1..8) */
  int32_t fp64_refine;   /* 1: stage 2 in FP64 when stage 1 runs in FP32 */
  double lambda0, lambda_min, lambda_max;  /* LM damping: start, floor, ceiling */
  double dup_eps;        /* SelectTop near-duplicate radius (infinity norm, rad) */
  int32_t k_seed;        /* path following: > 0 treats u_seed as per-waypoint IK seeds, runs this
                            many plain IK iterations per (seed, waypoint) and assembles one path
                            per seed from the waypoint solutions (Sec. IV-B); 0 = u_seed are paths */
} cr_opts;

/* ------------------------------------------------------------------------- */

/* Forward kinematics, Sec. III-A eq. (1)-(3) with the tendon map of eq. (4).
 * B configurations u[3n][ld] [device] -> per segment i:
 *   arc[3n][ld]    (kappa_i, phi_i, L_i): curvature 1/m, bending-plane azimuth in
 *                  [0, 2 pi) (0 when straight), arc length;  [device] or NULL
 *   frames[12n][ld] pose T_{0,i} of the tip of segment i (base frame at the
 *                  origin, backbone leaving along +z);  [device] or NULL
 *   pts[3nK][ld]   backbone points at arc fraction k/K, k = 1..K, component
 *                  c = 3*(i*K + k-1) + xyz;  [device] or NULL
 * The common mode of each segment's three tendons does not move the robot.
 * FP32 frames are re-orthonormalised in FP64 before they are written.
 * Errors: CR_EINVAL for a bad robot, B < 0, ld < B, u == NULL. */
cr_status cr_fk(const cr_robot* robot, int64_t B, const void* u, int64_t ld, void* arc,
                void* frames, void* pts, cr_dtype dtype, hipStream_t stream);

/* Penalised cost (eq. 17) and its gradient for a batch of seeds, with the task
 * objective of `kind` (IK eq. 8, path eq. 16, trajectory eq. 11) and the bound,
 * clearance, smoothness and endpoint penalties of eq. (9)-(15).
 *   P problems, S seeds each, H+1 waypoints per seed (H = 0 for IK).
 *   task  [device] IK: T_target[12][P]; PATH: T_ref[12][(H+1)*P] at column
 *         p*(H+1)+t; TRAJ: [6n][P], u_start (c < 3n) then u_goal.
 *   u     [device] [3n][(H+1)*S*P], column (p*S + s)*(H+1) + t.
 *   cost  [device] [S*P], column p*S + s: 1/2 sum of squared residuals.
 *   grad  [device] like u, or NULL for cost only: dC/du (zero-sum per segment,
 *         because the cost ignores each segment's common mode).
 *   grad_scale [device] [S*P] or NULL: grad of seed p*S + s is multiplied by
 *         grad_scale[p*S + s] (the upstream gradient of a backward pass).
 * All arrays, spheres included, are in `dtype`, and so is every step: with
 * CR_F32 the tendon map, the chained transforms, the backbone points, every
 * residual (pose, bounds, clearance, smoothness, endpoints) and the adjoint sweep
 * run in FP32 (a clearance hinge then carries the FP32 error of the point
 * positions, about 8 n 2^-24 sum(L) metres).  The gradient is formed by an
 * adjoint sweep over recomputed segment transforms (no stored Jacobian).
 * Errors: CR_EINVAL for bad shapes (H != 0 for IK, H < 1 for TRAJ, H > 255,
 * more than 512 spheres). */
cr_status cr_cost_grad(int32_t kind, const cr_robot* robot, const cr_spheres* spheres,
                       const cr_weights* weights, int64_t P, int32_t H, int32_t S,
                       const void* task, const void* u, void* cost, void* grad,
                       const void* grad_scale, cr_dtype dtype, hipStream_t stream);

/* SampleSeeds of Algorithm 1 (Sec. IV-B: initial configurations inside the
 * bounds; those that collide at once are discarded and drawn again), on the
 * device from a counter-based generator, so seeds need no host transfer.
 *   u_out [device, double] [3n][S*P], column p*S + s (the u_seed layout of the
 *         solve calls); attempts_out [device, int32] [S*P] or NULL.
 * Seed s of problem p reads the uniform stream U_j = word j mod 4 of
 * Philox4x64-10 (Salmon et al., SC 2011) at counter (j div 4, a, s, p) under key
 * (key0, key1), top 53 bits times 2^-53, for attempt a = 0, 1, ...: per segment,
 * triples x = u_max (2 U - 1) minus their mean until the zero-sum triple has
 * max |x| <= u_max and bending angle <= theta_max (at most 32 triples, else the
 * last one scaled onto the bounds); extensible robots then take the extension
 * L_min - L + (L_max - L_min) U, added to all three tendons.  An attempt is kept
 * if the configuration clears the spheres of problem p (and, with
 * self_collision, the robot itself) with margin 0 in FP64, or if it is attempt
 * max_attempts - 1.  attempts_out = attempts used, negated for a seed that still
 * collides.  A seed depends only on (key, p, s), not on P or S.  Spheres are
 * double, as for the solve calls.
 * Errors: CR_EINVAL for bad shapes or max_attempts outside 1..64. */
cr_status cr_sample_seeds(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t S,
                          uint64_t key0, uint64_t key1, int32_t max_attempts, double* u_out,
                          int32_t* attempts_out, hipStream_t stream);

/* Two-stage inverse kinematics, Algorithm 1: stage 1 runs k_init LM iterations
 * on every seed in `dtype`; SelectTop keeps n_final per problem; stage 2 runs
 * k_final LM iterations on those (in FP64 if fp64_refine or dtype is CR_F64);
 * the answer is the argmin of the final cost (ties: lowest seed index).  Stage 1
 * runs wholly in `dtype`, clearance and self-contact rows included; with CR_F32,
 * FP64 arithmetic is confined to stage 2 and to the assessment of the answer.
 *   T_target [device, double] [12][P];  u_seed [device, double] [3n][S*P],
 *   column p*S + s.
 *   u_out    [device, double] [3n][P]   zero-sum tendon displacements of q*
 *   err_out  [device, double] [2][P]    position error (m), rotation error (rad)
 *   status_out [device, int32] [P]      status bits
 *   ws/ws_bytes [device] scratch of at least cr_solve_ik_workspace() bytes,
 *   256-byte aligned (CR_EINVAL otherwise; hipMalloc's blocks are), or NULL/0
 *   to let the library allocate and free it stream-ordered.
 * Calls that share one workspace must not overlap. */
cr_status cr_solve_ik(const cr_robot* robot, const cr_spheres* spheres, int64_t P,
                      const void* T_target, int32_t S, const void* u_seed,
                      const cr_weights* weights, const cr_opts* opts, void* u_out, void* err_out,
                      int32_t* status_out, void* ws, size_t ws_bytes, cr_dtype dtype,
                      hipStream_t stream);

/* Workspace bytes cr_solve_ik needs for these shapes (0 on invalid arguments). */
size_t cr_solve_ik_workspace(const cr_robot* robot, int64_t P, int32_t S, const cr_opts* opts,
                             cr_dtype dtype);

/* Bytes of the static scratch buffer of cr_solve_ik_static on each GPU (64 MiB). */
#define CR_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* cr_solve_ik for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as cr_solve_ik, with the same arguments except the workspace: its scratch
 * is a static device buffer of CR_STATIC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine); its first call on a device
 * looks up that device's buffer address, with that device current.  Runs on the
 * current device; `stream` must belong to it.  The caller still owns T_target,
 * u_seed, u_out, err_out and status_out.
 * Every call on a GPU shares that GPU's buffer: calls that overlap on one GPU
 * (concurrent streams or host threads) race and must be serialised by the caller.
 * Errors: as cr_solve_ik, and CR_ENOMEM (nothing launched) when
 * cr_solve_ik_workspace() of these shapes exceeds CR_STATIC_SCRATCH_BYTES (the
 * 3-segment, 4096 x 256-seed, N_final = 8 FP32 solve needs 48 MB). */
cr_status cr_solve_ik_static(const cr_robot* robot, const cr_spheres* spheres, int64_t P,
                             const void* T_target, int32_t S, const void* u_seed,
                             const cr_weights* weights, const cr_opts* opts, void* u_out, void* err_out,
                             int32_t* status_out, cr_dtype dtype, hipStream_t stream);

/* Path following (eq. 16 with the trajectory constraints of eq. 12-15) for P
 * problems of H+1 waypoints, two-stage as in Algorithm 1 (Sec. IV-B): stage 1
 * runs k_init LM iterations over whole trajectories (block-pentadiagonal normal
 * equations, exact block Cholesky) on every seed in `dtype`; SelectTop keeps
 * n_final per problem ranked by total cost; stage 2 refines them in FP64; the
 * answer is the argmin of the final cost.
 *   T_ref  [device, double] [12][(H+1)*P], column p*(H+1) + t.
 *   u_seed [device, double] [3n][(H+1)*S*P], column (p*S + s)*(H+1) + t (the
 *          exploration stage's trajectories, e.g. per-waypoint IK, Sec. IV-B).
 *   u_out  [device, double] [3n][(H+1)*P]; err_out [2][P]: largest position /
 *          rotation error over the waypoints; status_out [P].
 *   spheres as in cr_cost_grad but double; ws/ws_bytes as in cr_solve_ik
 *   (size from cr_solve_traj_workspace).
 * Errors: CR_EINVAL for H > 255, S > 4096 or when (H+1) waypoints and the
 * spheres exceed 64 KiB of LDS per workgroup. */
cr_status cr_solve_path(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H,
                        const void* T_ref, int32_t S, const void* u_seed, const cr_weights* weights,
                        const cr_opts* opts, void* u_out, void* err_out, int32_t* status_out, void* ws,
                        size_t ws_bytes, cr_dtype dtype, hipStream_t stream);

/* Trajectory planning (eq. 11-15, endpoints penalised by eq. 17) between
 * u_start and u_goal, H >= 1; otherwise as cr_solve_path.
 *   u_start_goal [device, double] [6n][P]: u_start (c < 3n) then u_goal.
 *   err_out: largest endpoint position / rotation error against the start and
 *   goal poses; status adds CR_COLLISION for any penetrating backbone point. */
cr_status cr_solve_traj(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H,
                        const void* u_start_goal, int32_t S, const void* u_seed,
                        const cr_weights* weights, const cr_opts* opts, void* u_out, void* err_out,
                        int32_t* status_out, void* ws, size_t ws_bytes, cr_dtype dtype,
                        hipStream_t stream);

/* Workspace bytes cr_solve_path / cr_solve_traj need (0 on invalid arguments). */
size_t cr_solve_traj_workspace(const cr_robot* robot, int64_t P, int32_t H, int32_t S,
                               const cr_opts* opts, cr_dtype dtype);

/* ------------------------------------------------------------------------- */
/* Exploration stage of trajectory planning: probabilistic roadmap (PRM),      */
/* Algorithm 2.                                                                */
/* ------------------------------------------------------------------------- */

/* Roadmap and query parameters.  [host] */
typedef struct {
  int32_t n_nodes;       /* N roadmap samples per problem (ParallelSample), 1..2048 */
  int32_t k;             /* neighbours per node (ParallelConnect) and per query end
                            (ConnectToRoadmap), 1..32 */
  int32_t n_check;       /* interior configurations checked per straight motion, 0..64 */
  int32_t max_attempts;  /* SampleSeeds attempts per node, 1..64 */
  uint64_t key0, key1;   /* Philox key of the node draws */
} cr_prm_opts;

/* A neighbour-list slot without a neighbour. */
#define CR_PRM_NONE INT32_MIN

/* Offline roadmap of every problem's scene (Algorithm 2, ParallelSample and
 * ParallelConnect).  Configurations are tendon displacements u (3n numbers);
 * the distance of two is the Euclidean norm of their difference.  For P
 * problems, each with its own spheres (per_problem) or the shared ones:
 *  - node j of problem p is cr_sample_seeds' seed (key, p, j) with max_attempts;
 *    a node that still collides is discarded (attempts < 0);
 *  - every kept node lists its k nearest kept nodes (ties: lower index); the
 *    straight motion a -> b from the lower-indexed node is checked at the
 *    n_check configurations a + t_m (b - a), t_m = m / (n_check + 1),
 *    m = 1..n_check, with SampleSeeds' FP64 collision test (margin 0), endpoints
 *    not rechecked;
 *  - the roadmap is the undirected graph in which {i, j} is an edge when either
 *    lists the other with a free motion, weighted by their distance.
 * Outputs [device], B = N * P, column p * N + j:
 *   nodes    [3n][B] double    node configurations (zero-sum per segment)
 *   attempts [B] int32         SampleSeeds attempts, negative: node discarded
 *   nbr      [k][B] int32      slot s of node j at nbr[s * B + p * N + j]: the s-th
 *                              nearest kept node i (free motion), -1 - i (the motion
 *                              collides) or CR_PRM_NONE
 *   adj_off  [(N+1)*P] int32   CSR offsets of problem p at adj_off[p * (N + 1) + v],
 *                              relative to the problem's block
 *   adj      [2kN*P] int32     neighbours of node v of problem p at
 *                              adj[p * 2kN + adj_off[..v] .. p * 2kN + adj_off[..v+1]],
 *                              sorted by index
 *   adj_w    [2kN*P] double    the matching edge lengths
 * Distances and interpolations are formed with correctly rounded FP64 operations
 * in component order, without contraction.  Inextensible robots without self
 * contact and spheres only (the trajectory solve's scope).
 * Errors: CR_EINVAL for parameters outside the ranges above, P > 65535, polytopes;
 * CR_EUNSUPPORTED for extensible robots or self contact. */
cr_status cr_prm_build(const cr_robot* robot, const cr_spheres* spheres, int64_t P, const cr_prm_opts* prm,
                       double* nodes, int32_t* attempts, int32_t* nbr, int32_t* adj_off, int32_t* adj,
                       double* adj_w, hipStream_t stream);

/* Online queries (Algorithm 2, ConnectToRoadmap, Dijkstra, ResampleLinear): one
 * (start, goal) pair per problem on that problem's roadmap (cr_prm_build's
 * arrays, same P and prm), giving S initial trajectories of H+1 waypoints for
 * cr_solve_traj.
 *  - each end is joined to its k nearest kept nodes by the motions that pass the
 *    check above (starting at the end); the direct start-goal motion is an edge
 *    too when it passes;
 *  - Dijkstra over roadmap nodes 0..N-1, start N and goal N+1 settles nodes in
 *    order of (distance, index), relaxes on strict improvement and stops when
 *    the goal settles;
 *  - ResampleLinear: waypoint t (0 < t < H) lies at arc length s_m t / H along the
 *    path's polyline (s_i = the distance of the i-th path node), linearly
 *    interpolated in the first segment that reaches it; waypoint 0 is the start,
 *    H the goal; start and goal not connected: the straight line;
 *  - seed 0 is that trajectory; seed s >= 1 adds bump[.][column of s] (if bump is
 *    not NULL) and scales each (waypoint, segment) by min(1, u_max / max_j |u_j|).
 * linear = 1 skips the roadmap (the roadmap arrays may be NULL): the straight line
 * with the same perturbations (the linear initializer of Sec. V-C).
 *   u_start_goal [device, double] [6n][P]: start (c < 3n) then goal
 *   bump         [device, double] [3n][(H+1)*S*P] or NULL
 *   u_seed_out   [device, double] [3n][(H+1)*S*P], column (p*S + s)*(H+1) + t,
 *                the layout of cr_solve_traj's u_seed
 *   n_path_out   [device, int32] [P]: roadmap nodes on the path, -1 when start and
 *                goal are not connected (0 also for the direct motion and linear)
 *   path_out     [device, int32] [N+2][P] or NULL: node t of problem p's path at
 *                t * P + p (N = start, N + 1 = goal), -1 after the goal
 * Errors: as cr_prm_build, and CR_EINVAL for H outside 1..255 or S outside 1..4096. */
cr_status cr_prm_query(const cr_robot* robot, const cr_spheres* spheres, int64_t P, const cr_prm_opts* prm,
                       const double* nodes, const int32_t* attempts, const int32_t* adj_off, const int32_t* adj,
                       const double* adj_w, const double* u_start_goal, int32_t H, int32_t S, const double* bump,
                       int32_t linear, double* u_seed_out, int32_t* n_path_out, int32_t* path_out,
                       hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Uneven batches.                                                             */
/* ------------------------------------------------------------------------- */

/* One problem of an uneven batch ([host] table).  Every problem has its own
 * task kind, robot, horizon, seed count and spheres; its arrays are blocks at
 * element offsets into the packed [device, double] arrays of the call:
 *   task  IK: 12 values (3x4 row-major target pose, Sec. III-B);
 *         PATH: [12][H+1] (row r, waypoint t at task_off + r*(H+1) + t);
 *         TRAJ: [6n] (start then goal tendon displacements).
 *   seeds [3n][S*(H+1)] (row r, seed s, waypoint t at seed_off + r*S*(H+1) + s*(H+1) + t).
 *   spheres [4][n_sph] (component c of sphere m at sph_off + c*n_sph + m).
 *   output [3n][H+1] (row r, waypoint t at out_off + r*(H+1) + t).
 * Errors and status of problem i go to err_out[i], err_out[P + i], status_out[i]. */
typedef struct {
  int32_t kind;   /* cr_kind */
  int32_t robot;  /* index into the robots array */
  int32_t H;      /* IK: 0; PATH: 0..255; TRAJ: 1..255 */
  int32_t S;      /* 1..4096 seeds */
  int32_t n_sph;  /* 0..512 spheres */
  int32_t pad;
  int64_t task_off, seed_off, sph_off, out_off;
} cr_problem;

enum { CR_BATCH_GRAPH = 1, CR_BATCH_PERSISTENT = 2 }; /* cr_solve_batch flags */

/* Solves an uneven batch of P problems (Algorithm 1 for each, the same stages as
 * cr_solve_ik / cr_solve_path / cr_solve_traj).  A native scheduler groups the
 * problems by (kind, robot), orders each group longest-first by estimated work,
 * uploads one problem table per group and launches every group's ragged solve;
 * groups run concurrently on library-owned streams forked from `stream` and
 * joined back into it.
 *   robots [host] [n_robots]; probs [host] [P];
 *   weights, opts [host] [3], indexed by cr_kind;
 *   task, u_seed, sph, u_out [device, double] packed arrays (see cr_problem);
 *   err_out [device, double] [2][P]; status_out [device, int32] [P];
 *   ws/ws_bytes: at least cr_solve_batch_workspace() bytes, 256-byte aligned
 *   (required with CR_BATCH_GRAPH), or NULL/0 to let the library allocate
 *   stream-ordered.
 * flags & CR_BATCH_GRAPH: the whole launch sequence is captured once into a
 * hipGraph, cached by the call's arguments (table contents, pointers, options)
 * and replayed on later identical calls.  The cache owns the graphs and their
 * pinned table copies until the process ends.
 * flags & CR_BATCH_PERSISTENT: IK stage 1 of each group runs as one persistent
 * kernel that takes 64-seed tiles of all its problems from a device queue and
 * performs SelectTop inside the same launch, in the last workgroup to finish
 * a problem's tiles (no separate selection launch).  Results are identical
 * to the default launch sequence.
 * Errors: CR_EINVAL for a malformed table (kind, robot index, H, S, n_sph out of
 * range, negative offsets); array extents cannot be checked and are the
 * caller's responsibility.  Calls sharing a workspace must not overlap. */
cr_status cr_solve_batch(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P,
                         const void* task, const void* u_seed, const void* sph, const cr_weights* weights,
                         const cr_opts* opts, void* u_out, void* err_out, int32_t* status_out, void* ws,
                         size_t ws_bytes, cr_dtype dtype, int32_t flags, hipStream_t stream);

/* Workspace bytes of cr_solve_batch for this table (0 on invalid arguments). */
size_t cr_solve_batch_workspace(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P,
                                const cr_opts* opts, cr_dtype dtype);

/* SelectTop of Algorithm 1 on given candidates, per problem: order by e
 * ascending (ties: lower index; failed candidates never kept), greedily keep
 * candidates, a candidate within dup_eps (infinity norm over nz coordinates) of
 * a kept one replaces it iff its pen is strictly lower and is skipped otherwise;
 * if fewer than n_final remain, skipped ones refill in sorted order; -1 marks
 * an empty slot.
 *   z [device] [nz][S*P]; e, pen [device] [S*P]; failed [device, int32] [S*P]
 *   or NULL; idx_out [device, int32] [n_final][P] (seed index within the problem).
 * Errors: CR_EINVAL if S > 4096, n_final < 1 or n_final > 64. */
cr_status cr_select_top(int64_t P, int32_t S, int32_t nz, const void* z, const void* e,
                        const void* pen, const int32_t* failed, int32_t n_final, double dup_eps,
                        int32_t* idx_out, cr_dtype dtype, hipStream_t stream);

/* Comparison baseline: the plain per-problem FP32 IK solve the fused solver is
 * measured against.  The same Algorithm 1, iteration counts and LM rules as
 * cr_solve_ik, FP32 throughout (stage 2 included), run one problem after another
 * with a separate kernel per step: residuals and Jacobian by forward-mode dual
 * numbers (no adjoint), normal equations, damped Cholesky step, one kernel per
 * line-search trial and one per accept test, SelectTop, argmin; every
 * intermediate passes through HBM; no graph.  Arguments as cr_solve_ik (dtype
 * fixed to FP32); ws (256-byte aligned) at least S * (3n + 2)(2n + 6) * 4 +
 * 64 KiB bytes is always enough, or NULL/0 to let the library allocate. */
cr_status cr_baseline_solve_ik(const cr_robot* robot, const cr_spheres* spheres, int64_t P, const void* T_target,
                               int32_t S, const void* u_seed, const cr_weights* weights, const cr_opts* opts,
                               void* u_out, void* err_out, int32_t* status_out, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/* The plain per-problem FP32 comparison solve for path following and trajectory
 * planning: Algorithm 1 with the iteration counts and LM rules of cr_solve_path /
 * cr_solve_traj, but one problem at a time (its S trajectories), FP32 throughout
 * (stage 2 included), a separate kernel per step with every intermediate in HBM,
 * each waypoint's rows (pose, bounds, clearance of every backbone point against
 * every sphere, no culls) differentiated by forward-mode dual numbers, the
 * coupling rows assembled from the lifts' and tip positions' derivatives, and the
 * block-banded normal equations factored by one thread per trajectory.  The final
 * choice and its FP64 assessment are those of cr_solve_path / cr_solve_traj.
 * Arguments, layouts and outputs as cr_solve_path / cr_solve_traj (no dtype;
 * 1 <= S <= 4096).  ws: cr_baseline_traj_workspace() bytes, 256-byte aligned,
 * or NULL to allocate stream-ordered.  For timing against the fused solver; not used by it. */
cr_status cr_baseline_solve_path(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H,
                                 const void* T_ref, int32_t S, const void* u_seed, const cr_weights* weights,
                                 const cr_opts* opts, void* u_out, void* err_out, int32_t* status_out, void* ws,
                                 size_t ws_bytes, hipStream_t stream);
cr_status cr_baseline_solve_traj(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H,
                                 const void* u_start_goal, int32_t S, const void* u_seed,
                                 const cr_weights* weights, const cr_opts* opts, void* u_out, void* err_out,
                                 int32_t* status_out, void* ws, size_t ws_bytes, hipStream_t stream);
size_t cr_baseline_traj_workspace(const cr_robot* robot, int32_t H, int32_t S, const cr_opts* opts);

/* ------------------------------------------------------------------------- */
/* Instrumentation (benchmarks).                                               */
/* ------------------------------------------------------------------------- */

/* Stage timing of cr_solve_ik.  While enabled, every solve records HIP events on
 * its own stream around its four stages (stage 1, SelectTop, stage 2, final
 * argmin).  cr_timing_read() waits for the recorded calls, writes the summed
 * milliseconds per stage to stage_ms[4] and the number of calls, and clears the
 * record.  Enabling (or disabling) also clears it.  Process-wide state: one
 * benchmark at a time. */
void cr_timing_enable(int32_t on);
cr_status cr_timing_read(double* stage_ms, int64_t* n_calls);

/* Launch autotuning of the uneven-batch scheduling (a library-owned cache per
 * device).  The IK stage-1 kernels (uniform and table-driven) and the trajectory
 * normal-equation kernel are each compiled for three occupancy targets (the
 * minimum waves per SIMD their register allocation must allow).  The variants
 * compute the same formulas, but the compiler may contract different products
 * into fused multiply-adds under different register budgets, so FP32 results can
 * differ between variants in the last bits; each variant is deterministic, and a
 * cached choice reproduces the tuning call's results exactly.  While enabled, the
 * first FP32 launch of a key (kernel, segments, launch size rounded up to a power
 * of two, device) that is not being captured into a graph times each target three
 * times alone on the device (the call first waits for all queued device work, then
 * synchronises on the timing events) and later launches of the key use the one
 * with the shortest time.  Disabled (the default), or under capture with no
 * cached choice, the compiler's own target runs.  The FP64 IK stage 2 of robots
 * without clearance rows is tuned the same way over its lanes per kept candidate
 * (1, 2 or 4: the lanes of a candidate try that many line-search step lengths at
 * once and take the sequential search's choice, so its results do not depend on
 * the variant; FP32 and FP64 stage 1 alike); untuned, it takes the width that
 * gives each of the chip's 1024 SIMDs at most one wave.
 *   cr_autotune_enable(on): switch tuning on or off (the cache is kept).
 *   cr_autotune_clear():    forget every cached choice.
 *   cr_autotune_force(v):   run variant v (0: the compiler's own target, 1 and 2:
 *     the two tighter targets; IK stage 2: 2^v lanes per candidate) for every
 *     tunable kernel, tuning or not; v < 0 returns to normal operation.
 *   cr_autotune_report(buf, cap): text, one line per cached key (chosen target and
 *     the milliseconds of each), written to buf [host] when buf != NULL, truncated
 *     to cap - 1 bytes and NUL-terminated; returns the full length.
 * Process-wide state, guarded by a mutex. */
void cr_autotune_enable(int32_t on);
void cr_autotune_clear(void);
void cr_autotune_force(int32_t variant);
int64_t cr_autotune_report(char* buf, int64_t cap);

/* Algorithmic operation count of the IK stage-1 kernel, measured by replaying the
 * kernel's own arithmetic on the host with an op-counting scalar over n sample
 * seeds (k_init iterations plus the final evaluation each).
 *   T_target [host] [n][12] (pose of each sample's problem), u_seed [host] [n][3n].
 *   out [host] [8]: per seed {total flops, add/sub/mul, div, sqrt, sin/cos/atan2,
 *   line-search trials}, then the flops of one normal-equation evaluation and of
 *   one cost evaluation (first sample).  An FMA counts 2; div, sqrt and each
 *   transcendental count 1.  Runs on the calling thread; no device work. */
cr_status cr_ik_flop_tally(const cr_robot* robot, const cr_weights* weights, const cr_opts* opts, int64_t n,
                           const double* T_target, const double* u_seed, double* out);

/* Calibration of the vector-ALU accounting: launches `blocks` workgroups of 256
 * lanes, each lane running `iters` rounds over independent chains of one
 * instruction per chain and round: kind 0 v_fma_f32 (16 chains), 1 v_rcp_f32,
 * 2 v_fma_f32 on every chain plus v_rcp_f32 on every fourth, 3 v_fma_f64,
 * 4 v_add_f32, 5 v_mul_f32, 6 v_fma_f32 over 32 chains, 7 ten v_fma_f32, four
 * v_mul_f32 and two v_add_f32 per round, 8 and 9 as 0 with only the first 32 or
 * 16 lanes of every wave active.  The known instruction count per wave
 * against the measured duration gives the issue rate the SIMDs reach, and against
 * the SQ_INSTS_VALU* counters what those count.  out [device] receives blocks *
 * 256 floats.  CR_EINVAL for kind not in 0..9, blocks not in 1..2^20, iters < 1
 * or out == NULL. */
cr_status cr_calib_valu(int32_t kind, int64_t blocks, int32_t iters, float* out, hipStream_t stream);

/* Text for a status code, and the thread's last error message. */
const char* cr_status_string(cr_status s);
const char* cr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CR_SOLVER_H */
