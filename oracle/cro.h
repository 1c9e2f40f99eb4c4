/*
 * cro.h -- plain FP64 CPU oracle for CR-Solver (arXiv 2607.11340).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, scalar, single-threaded
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the GPU library.
 *
 * Conventions (all arrays are row-major C arrays of double, item-major):
 *   u    tendon displacements of one configuration, u[3*i + j] = length change of
 *        tendon j (at angle alpha_j = 2*pi*j/3) in segment i relative to L_i
 *        (Sec. III-B, eq. 4).
 *   z    coordinates of one configuration (the iterate of the solver), c per
 *        segment: z[c*i] = a_i = theta_i cos phi_i, z[c*i+1] = b_i = theta_i sin phi_i,
 *        and for extensible robots (c = 3) z[3*i+2] = e_i = mean_j u_ij, the change
 *        of the segment's length (L_i = L[i] + e_i); c = 2 otherwise.
 *   T    a pose as 12 doubles, 3x4 row-major [R | p].
 * A trajectory (kinds PATH/TRAJ) stores H+1 configurations back to back.
 */
#ifndef CRO_H
#define CRO_H
#include <stdint.h>

#define CRO_MAX_SEG 6
#define CRO_MAX_DIR (3 * CRO_MAX_SEG)

enum { CRO_IK = 0, CRO_PATH = 1, CRO_TRAJ = 2 };
enum {
  CRO_SOLVED = 1,
  CRO_LIMIT_VIOLATION = 2,
  CRO_COLLISION = 4,
  CRO_NONFINITE = 8,
  CRO_NOT_CONVERGED = 16
};

typedef struct {
  int32_t n_seg;       /* n, 1..CRO_MAX_SEG */
  int32_t pts_per_seg; /* K backbone sample points per segment (collision) */
  double L[CRO_MAX_SEG];     /* arc length of each segment, m */
  double r[CRO_MAX_SEG];     /* tendon routing radius r_c of each segment, m */
  double u_max[CRO_MAX_SEG]; /* bound on |tendon displacement|, m */
  double theta_max;          /* bound on each bending angle theta_i, rad */
  int32_t extensible;        /* 0: inextensible, the common mode of a segment's tendons is
                                ignored (eq. 4 with L fixed); 1: the common mode is the
                                segment's extension, L_i = L[i] + mean_j u_ij (Sec. V-B) */
  double L_min[CRO_MAX_SEG]; /* extensible: bounds on each segment length (eq. 9), m */
  double L_max[CRO_MAX_SEG];
  int32_t self_collision;    /* 1: backbone points of non-adjacent segments (|i - j| >= 2)
                                must keep r_i + r_j apart (eq. 10, self contact), with the
                                clearance penalty and margin of the obstacles */
} cro_robot;

typedef struct {
  double w_pos, w_rot;   /* pose residual weights */
  double rho_lim;        /* tendon-limit (and velocity/acceleration hinge) penalty */
  double rho_curv;       /* bending-angle limit penalty */
  double rho_coll;       /* obstacle penetration penalty */
  double margin;         /* safety margin delta, m */
  double rho_eq;         /* trajectory endpoint equality penalty */
  double w_len;          /* trajectory tip path-length weight */
  double w_vel, w_acc;   /* tendon velocity / acceleration smoothness weights */
  double v_max, a_max;   /* tendon velocity / acceleration bounds (INFINITY = off) */
  double dt;             /* time step */
} cro_weights;

typedef struct {
  int32_t n_final, k_init, k_final, ls_max;
  double lambda0, lambda_min, lambda_max, dup_eps;
  int32_t k_seed; /* PATH: > 0 builds the path seeds by per-waypoint IK (cro_path_seeds) */
} cro_opts;

typedef struct {
  int32_t kind;          /* CRO_IK, CRO_PATH, CRO_TRAJ */
  int32_t H;             /* horizon: H+1 waypoints (0 for IK) */
  const double* task;    /* IK: T[12]; PATH: T[(H+1)*12]; TRAJ: u_start[3n], u_goal[3n] */
  int32_t n_sph;         /* number of spheres */
  const double* sph;     /* [n_sph][4]: cx, cy, cz, radius */
  int32_t n_poly;        /* number of convex polytopes (IK only) */
  int32_t n_planes;      /* planes per polytope */
  const double* planes;  /* [n_poly][n_planes][4]: unit normal n and offset d of the
                            half-space n.x <= d; a polytope is the intersection of its
                            half-spaces (unused planes: n = 0, d large) */
} cro_problem;

#ifdef __cplusplus
extern "C" {
#endif

/* coordinates per segment: 3 for extensible robots, else 2 */
int cro_ncoord(const cro_robot* rb);

/* tendon displacements -> coordinates z, and the lift back (zero-sum per segment
 * when inextensible; with mean e_i when extensible) */
void cro_u_to_z(const cro_robot* rb, const double* u, double* z);
void cro_z_to_u(const cro_robot* rb, const double* z, double* u);

/* Forward kinematics of one configuration u[3n].
 * arc[3n]: (kappa, phi, L) per segment; frames[12n] or NULL: T_{0,i} of each
 * segment tip; pts[3nK] or NULL: backbone points, point k=1..K of segment i at
 * index (i*K + k-1)*3.  Returns 0. */
int cro_fk(const cro_robot* rb, const double* u, double* arc, double* frames, double* pts);

/* Penalised cost (eq. 17) of one seed of one problem, with u[(H+1)*3n].
 * grad_u (same shape) receives dC/du when non-NULL. */
double cro_cost(const cro_robot* rb, const cro_weights* w, const cro_problem* pb,
                const double* u, double* grad_u);

/* Residual vector r and dense Jacobian J = dr/dz ([m][(H+1)*c*n]) at z.
 * Returns the number of residual rows m, or -1 if it would exceed cap_rows. */
int cro_residuals(const cro_robot* rb, const cro_weights* w, const cro_problem* pb,
                  const double* z, double* r, double* J, int cap_rows);

/* Pose error of configuration z against pose T (eq. 18 and its parts):
 * out[0] = ||log(T_ee^-1 T)||_2, out[1] = position error (m), out[2] = rotation angle (rad). */
void cro_pose_error(const cro_robot* rb, const double* z, const double* T, double* out);

/* k Levenberg-Marquardt iterations with backtracking line search on one seed.
 * z and *lambda are updated in place.  Returns 1 if the seed failed (non-finite cost). */
int cro_lm(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, const cro_opts* o,
           double* z, double* lambda, int iters, double* cost_out, int* trials_out);

/* Cholesky solve of M x = y for symmetric positive definite M (N x N, lower triangle
 * read) with half bandwidth bw.  x holds y on entry.  Returns 0, or -1 on a
 * non-positive pivot.  M is overwritten by its factor. */
int cro_chol_solve(int N, int bw, double* M, double* x);

/* SelectTop of Algorithm 1: indices of n_final candidates out of S. */
void cro_select_top(int S, int nz, const double* z, const double* e, const double* pen,
                    const int32_t* failed, int n_final, double dup_eps, int32_t* idx_out);

/* Exploration stage of path following (Sec. IV-B): IK at every reference
 * waypoint from every seed, then one path per seed assembled from the waypoint
 * solutions.  u_seed[S][(H+1)*3n] are the IK seeds (seed s, waypoint t);
 * k iterations of the plain method run per (s, t) against the waypoint's pose
 * (with the problem's spheres).  Path s starts at the solution of seed s at
 * waypoint 0; each later waypoint takes, among its S solutions that pass the
 * success test (1 mm, 1 degree, bounds, no penetration), the one nearest in
 * the infinity norm over z to the path's previous waypoint (ties: lower seed);
 * if none passes, the nearest finite one; if none is finite, the previous
 * waypoint's z again.  z_out[S][(H+1)*c*n]. */
void cro_path_seeds(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, const cro_opts* o, int S,
                    const double* u_seed, int k, double* z_out);

/* Two-stage solve of one problem from S seeds u_seed[S][(H+1)*3n]
 * (Algorithm 1 for IK; the same template for PATH and TRAJ).
 * u_out[(H+1)*3n], err_out[2] (position m, rotation rad), *status (bits),
 * *best_idx (winning seed), *best_cost.  Returns 0, or -1 on bad arguments. */
int cro_solve(const cro_robot* rb, const cro_weights* w, const cro_problem* pb,
              const cro_opts* o, int S, const double* u_seed, double* u_out,
              double* err_out, int32_t* status, int32_t* best_idx, double* best_cost);

/* Philox4x64-10 counter-based generator (Salmon et al., SC 2011): out = the
 * four 64-bit words for counter ctr under key. */
void cro_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Triples drawn per segment before the bound is enforced by scaling. */
#define CRO_SEED_TRIPLES 32

/* SampleSeeds of Algorithm 1 for seed s of problem p (Sec. IV-B: inside the
 * bounds, seeds that collide at once are discarded).  Attempt a = 0, 1, ...
 * reads the uniform stream U_j = word j mod 4 of Philox4x64-10 at counter
 * (j div 4, a, s, p) under key, top 53 bits times 2^-53.  Per segment, in
 * order: triples x = u_max (2 U - 1) minus their mean until the zero-sum triple
 * has max |x| <= u_max and bending angle <= theta_max (at most CRO_SEED_TRIPLES
 * triples, else the last one scaled onto the bounds); extensible robots then take
 * the extension e = L_min - L + (L_max - L_min) U and every tendon adds e.  The
 * attempt is kept if it clears the spheres and, with self contact, the robot
 * itself (margin 0), or if it is attempt max_attempts - 1.  u[3n] receives the
 * seed; returns the number of attempts used, negated if the seed still collides. */
int32_t cro_sample_seed(const cro_robot* rb, const double* sph, int n_sph, const uint64_t key[2], int64_t p,
                        int32_t s, int32_t max_attempts, double* u);

/* Smallest clearance of configuration u[3n] against spheres sph[n_sph][4]
 * (x, y, z, radius) and, with self contact, the robot itself (eq. 10 with
 * margin 0): negative iff the configuration collides; INFINITY when there is
 * nothing to clear. */
double cro_contact_gap(const cro_robot* rb, const double* sph, int n_sph, const double* u);

#ifdef __cplusplus
}
#endif
#endif
