/*
 * cro.c -- plain FP64 CPU oracle for CR-Solver (arXiv 2607.11340).
 *
 * TEST INFRASTRUCTURE ONLY (see cro.h).  Scalar, single threaded, IEEE double,
 * built without fast-math and without FMA contraction.  Every derivative is
 * produced by forward-mode dual numbers pushed through the very formulas that
 * produce the values, so the Jacobian is exact by construction and shares no
 * hand-derived expression with the GPU library.
 *
 * Paper map:
 *   Sec. III-A eq. (1)-(3)   segment transform and chained forward kinematics
 *   Sec. III-B eq. (4)       tendon lengths <-> bending coordinates
 *   Sec. IV-A eq. (8)-(16)   IK, trajectory and path-following objectives/constraints
 *   Sec. IV-B eq. (17)       penalised cost
 *   Sec. IV-B Algorithm 1    two-stage beam search (SampleSeeds given by the caller,
 *                            ParallelOptimize, SelectTop, final argmin)
 *   Sec. IV-C                batched Levenberg-Marquardt with Cholesky solves
 *   Sec. V-B eq. (18)        SE(3) log pose error; success criterion
 */
#include "cro.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ND CRO_MAX_DIR
#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Dual numbers: value plus derivatives along nd directions.                   */
/* ------------------------------------------------------------------------- */

typedef struct {
  double v;
  double d[ND];
} dual;

static int nd = 0; /* live derivative directions of the current evaluation */

static dual dcon(double v) {
  dual r;
  r.v = v;
  for (int k = 0; k < nd; k++) r.d[k] = 0.0;
  return r;
}
static dual dvar(double v, int dir) {
  dual r = dcon(v);
  if (dir < nd) r.d[dir] = 1.0;
  return r;
}
static dual dadd(dual a, dual b) {
  dual r;
  r.v = a.v + b.v;
  for (int k = 0; k < nd; k++) r.d[k] = a.d[k] + b.d[k];
  return r;
}
static dual dsub(dual a, dual b) {
  dual r;
  r.v = a.v - b.v;
  for (int k = 0; k < nd; k++) r.d[k] = a.d[k] - b.d[k];
  return r;
}
static dual dneg(dual a) {
  dual r;
  r.v = -a.v;
  for (int k = 0; k < nd; k++) r.d[k] = -a.d[k];
  return r;
}
static dual dmul(dual a, dual b) {
  dual r;
  r.v = a.v * b.v;
  for (int k = 0; k < nd; k++) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
static dual dscale(double c, dual a) {
  dual r;
  r.v = c * a.v;
  for (int k = 0; k < nd; k++) r.d[k] = c * a.d[k];
  return r;
}
static dual dshift(dual a, double c) {
  a.v += c;
  return a;
}
static dual ddiv(dual a, dual b) {
  dual r;
  r.v = a.v / b.v;
  for (int k = 0; k < nd; k++) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
/* f(x) for a scalar function with value f and derivative df at x.v */
static dual dapply(dual x, double f, double df) {
  dual r;
  r.v = f;
  for (int k = 0; k < nd; k++) r.d[k] = df * x.d[k];
  return r;
}
static dual dsqrt(dual a) {
  double s = sqrt(a.v);
  return dapply(a, s, 0.5 / s);
}
static dual datan2(dual y, dual x) {
  dual r;
  double den = x.v * x.v + y.v * y.v;
  r.v = atan2(y.v, x.v);
  for (int k = 0; k < nd; k++) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) / den;
  return r;
}

/* 3-vectors and row-major 3x3 matrices of duals */
static void mat_mul(const dual* A, const dual* B, dual* C) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      dual s = dcon(0.0);
      for (int k = 0; k < 3; k++) s = dadd(s, dmul(A[3 * i + k], B[3 * k + j]));
      C[3 * i + j] = s;
    }
}
static void mat_vec(const dual* A, const dual* x, dual* y) {
  for (int i = 0; i < 3; i++) {
    dual s = dcon(0.0);
    for (int k = 0; k < 3; k++) s = dadd(s, dmul(A[3 * i + k], x[k]));
    y[i] = s;
  }
}
static void matT_vec(const dual* A, const dual* x, dual* y) {
  for (int i = 0; i < 3; i++) {
    dual s = dcon(0.0);
    for (int k = 0; k < 3; k++) s = dadd(s, dmul(A[3 * k + i], x[k]));
    y[i] = s;
  }
}
static void cross(const dual* a, const dual* b, dual* c) {
  dual t0 = dsub(dmul(a[1], b[2]), dmul(a[2], b[1]));
  dual t1 = dsub(dmul(a[2], b[0]), dmul(a[0], b[2]));
  dual t2 = dsub(dmul(a[0], b[1]), dmul(a[1], b[0]));
  c[0] = t0;
  c[1] = t1;
  c[2] = t2;
}
static dual dot3(const dual* a, const dual* b) {
  return dadd(dadd(dmul(a[0], b[0]), dmul(a[1], b[1])), dmul(a[2], b[2]));
}
/* [w]_x, the cross-product matrix */
static void skew(const dual* w, dual* S) {
  S[0] = dcon(0.0);
  S[1] = dneg(w[2]);
  S[2] = w[1];
  S[3] = w[2];
  S[4] = dcon(0.0);
  S[5] = dneg(w[0]);
  S[6] = dneg(w[1]);
  S[7] = w[0];
  S[8] = dcon(0.0);
}

/* ------------------------------------------------------------------------- */
/* Smooth scalar functions of s = theta^2 (so that theta = 0 is a regular     */
/* point), each returned with its s-derivative.                               */
/* ------------------------------------------------------------------------- */

/* Taylor series  sum_k (-s)^k / (2k+off)!  and its s-derivative.
 * off = 1: sin(x)/x, off = 2: (1 - cos x)/x^2, with s = x^2. */
static void trig_series(double s, int off, double* f, double* df) {
  double fact = 1.0;
  for (int m = 2; m <= off; m++) fact *= m;
  double sum = 0.0, dsum = 0.0, sk = 1.0, skm1 = 0.0;
  for (int k = 0; k < 9; k++) {
    double c = ((k & 1) ? -1.0 : 1.0) / fact;
    sum += c * sk;
    if (k > 0) dsum += k * c * skm1;
    skm1 = sk;
    sk *= s;
    fact *= (double)(2 * k + off + 1) * (double)(2 * k + off + 2);
  }
  *f = sum;
  *df = dsum;
}

/* B(s) = sin(theta)/theta */
static dual fam_B(dual s) {
  double f, df;
  if (s.v < 1e-2) {
    trig_series(s.v, 1, &f, &df);
  } else {
    double x = sqrt(s.v);
    f = sin(x) / x;
    df = (cos(x) - f) / (2.0 * s.v);
  }
  return dapply(s, f, df);
}
/* A(s) = (1 - cos theta)/theta^2 */
static dual fam_A(dual s) {
  double f, df;
  if (s.v < 1e-2) {
    trig_series(s.v, 2, &f, &df);
  } else {
    double x = sqrt(s.v), hs = sin(0.5 * x);
    double B = sin(x) / x;
    f = 2.0 * hs * hs / s.v;
    df = (0.5 * B - f) / s.v;
  }
  return dapply(s, f, df);
}

/* g(x) = asin(sqrt x)/sqrt x = theta/sin(theta) for x = sin^2(theta), theta < pi/2.
 * Series coefficients C(2k,k) / (4^k (2k+1)). */
static dual fam_asin_ratio(dual x) {
  double f, df;
  if (x.v < 1e-2) {
    double sum = 0.0, dsum = 0.0, xk = 1.0, xkm1 = 0.0, binom = 1.0, p4 = 1.0;
    for (int k = 0; k < 9; k++) {
      if (k > 0) {
        binom = binom * (double)(2 * k) * (double)(2 * k - 1) / ((double)k * (double)k);
        p4 *= 4.0;
      }
      double c = binom / (p4 * (double)(2 * k + 1));
      sum += c * xk;
      if (k > 0) dsum += k * c * xkm1;
      xkm1 = xk;
      xk *= x.v;
    }
    f = sum;
    df = dsum;
  } else {
    double y = sqrt(x.v);
    f = asin(y) / y;
    df = (1.0 / sqrt(1.0 - x.v) - f) / (2.0 * x.v);
  }
  return dapply(x, f, df);
}

/* gamma(q) = (1 - (theta/2) cot(theta/2)) / theta^2, q = theta^2, the coefficient of
 * [w]_x^2 in the inverse of the SE(3) left Jacobian V.
 * Series: gamma = sum_{k>=1} |B_2k| q^(k-1) / (2k)!  (Bernoulli numbers). */
static dual fam_gamma(dual q) {
  static const double bern_abs[7] = {1.0 / 6.0,    1.0 / 30.0,  1.0 / 42.0,
                                     1.0 / 30.0,   5.0 / 66.0,  691.0 / 2730.0,
                                     7.0 / 6.0};
  double f, df;
  if (q.v < 1e-2) {
    double sum = 0.0, dsum = 0.0, qk = 1.0, qkm1 = 0.0, fact = 2.0; /* (2k)! for k=1 */
    for (int k = 1; k <= 7; k++) {
      double c = bern_abs[k - 1] / fact;
      sum += c * qk;
      if (k > 1) dsum += (k - 1) * c * qkm1;
      qkm1 = qk;
      qk *= q.v;
      fact *= (double)(2 * k + 1) * (double)(2 * k + 2);
    }
    f = sum;
    df = dsum;
  } else {
    double th = sqrt(q.v), h = 0.5 * th / tan(0.5 * th);
    double sh = sin(0.5 * th);
    double dh_dth = 0.5 / tan(0.5 * th) - 0.25 * th / (sh * sh);
    f = (1.0 - h) / q.v;
    df = (-dh_dth / (2.0 * th) - f) / q.v;
  }
  return dapply(q, f, df);
}

/* ------------------------------------------------------------------------- */
/* Actuation model (Sec. III-B, eq. 4).                                        */
/* ------------------------------------------------------------------------- */

static double alpha_j(int j) { return 2.0 * PI * (double)j / 3.0; }

int cro_ncoord(const cro_robot* rb) { return rb->extensible ? 3 : 2; }

/* eq. (4) minus L_i:  u_ij = -r_c theta_i cos(alpha_j - phi_i) = -r_c (a cos alpha_j + b sin alpha_j).
 * Three tendons at 0, 120, 240 degrees are orthogonal in the sense
 * sum_j cos^2 = sum_j sin^2 = 3/2, sum_j cos sin = sum_j cos = sum_j sin = 0, so
 * projecting u on cos/sin inverts eq. (4) and ignores the common mode. */
void cro_u_to_z(const cro_robot* rb, const double* u, double* z) {
  int c = cro_ncoord(rb);
  for (int i = 0; i < rb->n_seg; i++) {
    double pc = 0.0, ps = 0.0;
    for (int j = 0; j < 3; j++) {
      pc += u[3 * i + j] * cos(alpha_j(j));
      ps += u[3 * i + j] * sin(alpha_j(j));
    }
    z[c * i] = -pc / (1.5 * rb->r[i]);
    z[c * i + 1] = -ps / (1.5 * rb->r[i]);
    /* extensible: the common mode is the change of the segment's length (the mean of
     * eq. 4 over the three tendons is L_i) */
    if (c == 3) z[c * i + 2] = (u[3 * i] + u[3 * i + 1] + u[3 * i + 2]) / 3.0;
  }
}

void cro_z_to_u(const cro_robot* rb, const double* z, double* u) {
  int c = cro_ncoord(rb);
  for (int i = 0; i < rb->n_seg; i++)
    for (int j = 0; j < 3; j++) {
      u[3 * i + j] = -rb->r[i] * (z[c * i] * cos(alpha_j(j)) + z[c * i + 1] * sin(alpha_j(j)));
      if (c == 3) u[3 * i + j] += z[c * i + 2];
    }
}

/* bending part of tendon j of segment i (zero-sum over j) */
static dual bend_dual(const cro_robot* rb, const dual* z, int i, int j) {
  int c = cro_ncoord(rb);
  return dscale(-rb->r[i], dadd(dscale(cos(alpha_j(j)), z[c * i]), dscale(sin(alpha_j(j)), z[c * i + 1])));
}

/* whole displacement of tendon j of segment i: bending part plus extension */
static dual lift_dual(const cro_robot* rb, const dual* z, int i, int j) {
  dual u = bend_dual(rb, z, i, j);
  return cro_ncoord(rb) == 3 ? dadd(u, z[3 * i + 2]) : u;
}

/* length of segment i */
static dual seg_len(const cro_robot* rb, const dual* z, int i) {
  return cro_ncoord(rb) == 3 ? dshift(z[3 * i + 2], rb->L[i]) : dcon(rb->L[i]);
}

/* ------------------------------------------------------------------------- */
/* Forward kinematics (Sec. III-A, eq. 1-3).                                   */
/* ------------------------------------------------------------------------- */

/* Transform of one constant-curvature arc with bending coordinates (a, b) and length L.
 * eq. (2): R = Z(phi) Y(theta) Z(-phi) is the rotation by theta about the in-plane
 * axis (-sin phi, cos phi, 0), i.e. exp([w]_x) with w = (-b, a, 0); by Rodrigues
 * R = I + B [w]_x + A [w]_x^2.
 * eq. (3): d = (L/theta) (cos phi (1-cos theta), sin phi (1-cos theta), sin theta)
 *          = L (A a, A b, B), which also covers the straight case theta = 0. */
static void arc_transform(dual a, dual b, dual L, dual* R, dual* d) {
  dual s = dadd(dmul(a, a), dmul(b, b));
  dual A = fam_A(s), B = fam_B(s);
  dual w[3] = {dneg(b), a, dcon(0.0)};
  dual W[9], W2[9];
  skew(w, W);
  mat_mul(W, W, W2);
  for (int k = 0; k < 9; k++) R[k] = dadd(dmul(B, W[k]), dmul(A, W2[k]));
  R[0] = dshift(R[0], 1.0);
  R[4] = dshift(R[4], 1.0);
  R[8] = dshift(R[8], 1.0);
  d[0] = dmul(L, dmul(A, a));
  d[1] = dmul(L, dmul(A, b));
  d[2] = dmul(L, B);
}

/* Chain T_{0,i} = T_{0,i-1} T_{i-1}^{i} (eq. 1) from the base frame (identity).
 * Rf[i], pf[i]: frame at the tip of segment i.  pts (optional): backbone points
 * at arc fraction sigma = k/K, k = 1..K, of each segment. */
static void fk_chain(const cro_robot* rb, const dual* z, dual (*Rf)[9], dual (*pf)[3], dual (*pts)[3]) {
  dual R[9], p[3];
  for (int k = 0; k < 9; k++) R[k] = dcon((k % 4 == 0) ? 1.0 : 0.0);
  for (int k = 0; k < 3; k++) p[k] = dcon(0.0);
  int K = rb->pts_per_seg, zc = cro_ncoord(rb);
  for (int i = 0; i < rb->n_seg; i++) {
    dual Li = seg_len(rb, z, i);
    if (pts) {
      for (int k = 1; k <= K; k++) {
        double sg = (double)k / (double)K;
        dual Rk[9], dk[3], q[3];
        arc_transform(dscale(sg, z[zc * i]), dscale(sg, z[zc * i + 1]), dscale(sg, Li), Rk, dk);
        mat_vec(R, dk, q);
        for (int c = 0; c < 3; c++) pts[i * K + k - 1][c] = dadd(p[c], q[c]);
      }
    }
    dual Ri[9], di[3], q[3], Rn[9];
    arc_transform(z[zc * i], z[zc * i + 1], Li, Ri, di);
    mat_vec(R, di, q);
    for (int c = 0; c < 3; c++) p[c] = dadd(p[c], q[c]);
    mat_mul(R, Ri, Rn);
    memcpy(R, Rn, sizeof(R));
    memcpy(Rf[i], R, sizeof(R));
    memcpy(pf[i], p, sizeof(p));
  }
}

int cro_fk(const cro_robot* rb, const double* u, double* arc, double* frames, double* pts) {
  int n = rb->n_seg, K = rb->pts_per_seg, zc = cro_ncoord(rb);
  double zz[CRO_MAX_DIR];
  dual z[CRO_MAX_DIR], Rf[CRO_MAX_SEG][9], pf[CRO_MAX_SEG][3];
  nd = 0;
  cro_u_to_z(rb, u, zz);
  for (int k = 0; k < zc * n; k++) z[k] = dcon(zz[k]);
  dual(*P)[3] = NULL;
  if (pts && K > 0) P = (dual(*)[3])malloc(sizeof(dual[3]) * (size_t)(n * K));
  fk_chain(rb, z, Rf, pf, P);
  for (int i = 0; i < n; i++) {
    double a = zz[zc * i], b = zz[zc * i + 1], th = sqrt(a * a + b * b);
    double ph = (th > 0.0) ? atan2(b, a) : 0.0;
    if (ph < 0.0) ph += 2.0 * PI;
    double Li = seg_len(rb, z, i).v;
    arc[3 * i] = th / Li;
    arc[3 * i + 1] = ph;
    arc[3 * i + 2] = Li;
    if (frames) {
      for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) frames[12 * i + 4 * r + c] = Rf[i][3 * r + c].v;
        frames[12 * i + 4 * r + 3] = pf[i][r].v;
      }
    }
  }
  if (P) {
    for (int m = 0; m < n * K; m++)
      for (int c = 0; c < 3; c++) pts[3 * m + c] = P[m][c].v;
    free(P);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* SE(3) logarithm (eq. 8, 16, 18).                                            */
/* ------------------------------------------------------------------------- */

/* (rho, w) = log(E) for E = [Re | te]; w = Log_SO3(Re), rho = V(w)^-1 te with
 * V^-1 = I - [w]_x / 2 + gamma(|w|^2) [w]_x^2.  Three algebraically equal forms
 * of w keep every branch well conditioned:
 *   cos >= 1/2      w = v * theta/sin(theta), theta/sin as a series in sin^2
 *   -0.9 <= cos     w = v * atan2(|v|, cos) / |v|
 *   cos < -0.9      w = theta * n, n from the symmetric part of Re (near pi)
 * where v = vee(Re - Re^T)/2 = sin(theta) n. */
static void log_se3(const dual* Re, const dual* te, dual* rho, dual* w) {
  dual c = dscale(0.5, dshift(dadd(dadd(Re[0], Re[4]), Re[8]), -1.0));
  dual v[3] = {dscale(0.5, dsub(Re[7], Re[5])), dscale(0.5, dsub(Re[2], Re[6])),
               dscale(0.5, dsub(Re[3], Re[1]))};
  if (c.v >= 0.5) {
    dual g = fam_asin_ratio(dot3(v, v));
    for (int k = 0; k < 3; k++) w[k] = dmul(v[k], g);
  } else if (c.v >= -0.9) {
    dual sn = dsqrt(dot3(v, v));
    dual ratio = ddiv(datan2(sn, c), sn);
    for (int k = 0; k < 3; k++) w[k] = dmul(v[k], ratio);
  } else {
    /* (Re + Re^T)/2 = c I + (1 - c) n n^T */
    dual nn[9];
    dual omc = dsub(dcon(1.0), c);
    for (int r = 0; r < 3; r++)
      for (int q = 0; q < 3; q++) {
        dual sym = dscale(0.5, dadd(Re[3 * r + q], Re[3 * q + r]));
        if (r == q) sym = dsub(sym, c);
        nn[3 * r + q] = ddiv(sym, omc);
      }
    int kk = 0;
    for (int k = 1; k < 3; k++)
      if (nn[4 * k].v > nn[4 * kk].v) kk = k;
    dual nk = dsqrt(nn[4 * kk]);
    dual n[3];
    for (int r = 0; r < 3; r++) n[r] = ddiv(nn[3 * r + kk], nk);
    dual sn = dot3(n, v);
    int flip = 0;
    if (sn.v < 0.0) {
      flip = 1;
    } else if (sn.v == 0.0) { /* theta = pi exactly: first nonzero component positive */
      for (int r = 0; r < 3; r++)
        if (n[r].v != 0.0) {
          flip = n[r].v < 0.0;
          break;
        }
    }
    if (flip) {
      for (int r = 0; r < 3; r++) n[r] = dneg(n[r]);
      sn = dneg(sn);
    }
    dual th = datan2(sn, c);
    for (int k = 0; k < 3; k++) w[k] = dmul(th, n[k]);
  }
  dual gam = fam_gamma(dot3(w, w));
  dual w1[3], w2[3];
  cross(w, te, w1);
  cross(w, w1, w2);
  for (int k = 0; k < 3; k++) rho[k] = dadd(dsub(te[k], dscale(0.5, w1[k])), dmul(gam, w2[k]));
}

/* log(T_ee^-1 T) for the tip frame (R, p) against a target pose T[12] (3x4 row-major). */
static void pose_log(const dual* R, const dual* p, const double* T, dual* rho, dual* w) {
  dual Rt[9], dp[3], Re[9], te[3];
  for (int r = 0; r < 3; r++) {
    for (int c = 0; c < 3; c++) Rt[3 * r + c] = dcon(T[4 * r + c]);
    dp[r] = dsub(dcon(T[4 * r + 3]), p[r]);
  }
  /* Re = R^T Rt, te = R^T (pt - p) */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      dual s = dcon(0.0);
      for (int k = 0; k < 3; k++) s = dadd(s, dmul(R[3 * k + i], Rt[3 * k + j]));
      Re[3 * i + j] = s;
    }
  matT_vec(R, dp, te);
  log_se3(Re, te, rho, w);
}

/* ------------------------------------------------------------------------- */
/* Residual sink: accumulates cost = 1/2 sum r^2, g = J^T r, H = J^T J and,   */
/* for tests, the dense rows of J.                                             */
/* ------------------------------------------------------------------------- */

typedef struct {
  int nz;      /* unknowns per waypoint (2n) */
  int N;       /* total unknowns (H+1)*nz */
  double cost;
  double* g;   /* [N] or NULL */
  double* Hm;  /* [N*N] or NULL */
  double* r;   /* captured residuals or NULL */
  double* J;   /* captured dense Jacobian rows [cap][N] or NULL */
  int rows, cap, overflow;
} sink;

typedef struct {
  int t;         /* waypoint the dual's directions belong to */
  double c;      /* coefficient */
  const dual* x; /* dual over that waypoint's z */
} term;

/* One residual row  r = scale * (sum_j c_j x_j.v)  or its hinge (see emit_hinge). */
static void emit_row(sink* s, double r, double jscale, int nt, const term* tm) {
  s->cost += 0.5 * r * r;
  int need = (s->g || s->Hm || s->J);
  if (!need) return;
  int cols[3 * ND];
  double jr[3 * ND];
  int m = 0;
  for (int j = 0; j < nt; j++)
    for (int k = 0; k < s->nz; k++) {
      int col = tm[j].t * s->nz + k;
      double val = jscale * tm[j].c * tm[j].x->d[k];
      int found = -1;
      for (int q = 0; q < m; q++)
        if (cols[q] == col) found = q;
      if (found >= 0) {
        jr[found] += val;
      } else {
        cols[m] = col;
        jr[m] = val;
        m++;
      }
    }
  if (s->g)
    for (int a = 0; a < m; a++) s->g[cols[a]] += jr[a] * r;
  if (s->Hm)
    for (int a = 0; a < m; a++)
      for (int b = 0; b < m; b++) s->Hm[(size_t)cols[a] * s->N + cols[b]] += jr[a] * jr[b];
  if (s->J) {
    if (s->rows >= s->cap) {
      s->overflow = 1;
    } else {
      double* row = s->J + (size_t)s->rows * s->N;
      for (int q = 0; q < s->N; q++) row[q] = 0.0;
      for (int a = 0; a < m; a++) row[cols[a]] += jr[a];
      s->r[s->rows] = r;
    }
  }
  s->rows++;
}

/* Plain row: r = scale * sum_j c_j x_j */
static void emit_lin(sink* s, double scale, int nt, const term* tm) {
  double v = 0.0;
  for (int j = 0; j < nt; j++) v += tm[j].c * tm[j].x->v;
  emit_row(s, scale * v, scale, nt, tm);
}

/* Hinge row (eq. 17, Pi_ineq is zero when satisfied):
 * r = scale * max(0, |sum_j c_j x_j| - bound); derivative 0 at and below the kink. */
static void emit_hinge(sink* s, double scale, double bound, int nt, const term* tm) {
  double v = 0.0;
  for (int j = 0; j < nt; j++) v += tm[j].c * tm[j].x->v;
  double viol = fabs(v) - bound;
  if (!(viol > 0.0)) return;
  emit_row(s, scale * viol, (v < 0.0) ? -scale : scale, nt, tm);
}

/* ------------------------------------------------------------------------- */
/* Cost of one seed (eq. 8-17).                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
  dual z[ND];
  dual R[9], p[3];             /* tip frame */
  dual u[3 * CRO_MAX_SEG];     /* lifted tendon displacements */
} waypoint;

static int is_finite_bound(double x) { return isfinite(x); }

/* Obstacle rows of one waypoint: each backbone point against each sphere,
 * g = |p - c| - R_s - r_i (body radius = tendon radius), r = sqrt(rho_coll) max(0, margin - g).
 * The value is checked first in plain double; only active pairs are differentiated. */
static void collision_rows(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, int t,
                           dual (*pts)[3], sink* s) {
  int n = rb->n_seg, K = rb->pts_per_seg;
  double sq = sqrt(w->rho_coll);
  for (int i = 0; i < n; i++)
    for (int k = 0; k < K; k++) {
      dual* P = pts[i * K + k];
      for (int m = 0; m < pb->n_sph; m++) {
        const double* S = pb->sph + 4 * m;
        double dx = P[0].v - S[0], dy = P[1].v - S[1], dz = P[2].v - S[2];
        double dist = sqrt(dx * dx + dy * dy + dz * dz);
        double gap = dist - S[3] - rb->r[i];
        if (!(w->margin - gap > 0.0)) continue;
        dual ddist;
        if (dist > 0.0) {
          dual q[3] = {dshift(P[0], -S[0]), dshift(P[1], -S[1]), dshift(P[2], -S[2])};
          ddist = dsqrt(dot3(q, q));
        } else { /* coincident: take the +z direction */
          ddist = dshift(P[2], -S[2]);
          ddist.v = 0.0;
        }
        dual viol = dsub(dcon(w->margin + S[3] + rb->r[i]), ddist);
        term tm = {t, 1.0, &viol};
        emit_lin(s, sq, 1, &tm);
      }
    }
}

/* Signed distance of point x to convex polytope j in half-space form: the largest
 * of n_f.x - d_f over its planes (exact inside the polytope and in the region of
 * each face outside it; below the distance near edges and corners outside).
 * *arg receives the plane of the first largest value. */
static double poly_sd(const cro_problem* pb, int j, const double* x, int* arg) {
  double s = -INFINITY;
  int a = 0;
  for (int f = 0; f < pb->n_planes; f++) {
    const double* P = pb->planes + 4 * ((size_t)j * pb->n_planes + f);
    double v = P[0] * x[0] + P[1] * x[1] + P[2] * x[2] - P[3];
    if (v > s) {
      s = v;
      a = f;
    }
  }
  if (arg) *arg = a;
  return s;
}

/* Polytope rows of one waypoint (convex obstacles, eq. 10 with the signed
 * distance above): gap = sd(p) - r_i, r = sqrt(rho_coll) max(0, margin - gap),
 * differentiated through the plane that attains the distance. */
static void polytope_rows(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, int t,
                          dual (*pts)[3], sink* s) {
  int n = rb->n_seg, K = rb->pts_per_seg;
  double sq = sqrt(w->rho_coll);
  for (int i = 0; i < n; i++)
    for (int k = 0; k < K; k++) {
      dual* P = pts[i * K + k];
      double x[3] = {P[0].v, P[1].v, P[2].v};
      for (int j = 0; j < pb->n_poly; j++) {
        int f;
        double gap = poly_sd(pb, j, x, &f) - rb->r[i];
        if (!(w->margin - gap > 0.0)) continue;
        const double* Q = pb->planes + 4 * ((size_t)j * pb->n_planes + f);
        dual sd = dshift(dadd(dadd(dscale(Q[0], P[0]), dscale(Q[1], P[1])), dscale(Q[2], P[2])), -Q[3]);
        dual viol = dsub(dcon(w->margin + rb->r[i]), sd);
        term tm = {t, 1.0, &viol};
        emit_lin(s, sq, 1, &tm);
      }
    }
}

/* Self-contact rows of one waypoint (eq. 10): every pair of backbone points p, q
 * of segments i and j >= i + 2, gap = |p - q| - r_i - r_j,
 * r = sqrt(rho_coll) max(0, margin - gap). */
static void self_rows(const cro_robot* rb, const cro_weights* w, int t, dual (*pts)[3], sink* s) {
  int n = rb->n_seg, K = rb->pts_per_seg;
  double sq = sqrt(w->rho_coll);
  for (int i = 0; i < n; i++)
    for (int j = i + 2; j < n; j++)
      for (int k = 0; k < K; k++)
        for (int l = 0; l < K; l++) {
          dual* P = pts[i * K + k];
          dual* Q = pts[j * K + l];
          double dx = Q[0].v - P[0].v, dy = Q[1].v - P[1].v, dz = Q[2].v - P[2].v;
          double dist = sqrt(dx * dx + dy * dy + dz * dz);
          double gap = dist - rb->r[i] - rb->r[j];
          if (!(w->margin - gap > 0.0)) continue;
          dual ddist;
          if (dist > 0.0) {
            dual q[3] = {dsub(Q[0], P[0]), dsub(Q[1], P[1]), dsub(Q[2], P[2])};
            ddist = dsqrt(dot3(q, q));
          } else { /* coincident: take the +z direction */
            ddist = dsub(Q[2], P[2]);
            ddist.v = 0.0;
          }
          dual viol = dsub(dcon(w->margin + rb->r[i] + rb->r[j]), ddist);
          term tm = {t, 1.0, &viol};
          emit_lin(s, sq, 1, &tm);
        }
}

/* groups of cost terms, so that the collision penalty alone can be evaluated */
enum { T_TASK = 1, T_LIMITS = 2, T_COLL = 4, T_SMOOTH = 8, T_LEN = 16, T_ENDS = 32, T_ALL = 63 };

static double eval_terms(const cro_robot* rb, const cro_weights* w, const cro_problem* pb,
                         const double* z, sink* s, int terms) {
  int n = rb->n_seg, zc = cro_ncoord(rb), nz = zc * n, H = pb->H, K = rb->pts_per_seg;
  int derive = (s->g || s->Hm || s->J);
  nd = derive ? nz : 0;
  s->cost = 0.0;
  s->rows = 0;
  waypoint* wp = (waypoint*)malloc(sizeof(waypoint) * (size_t)(H + 1));
  dual(*pts)[3] = NULL;
  if ((pb->n_sph > 0 || pb->n_poly > 0 || rb->self_collision) && K > 0)
    pts = (dual(*)[3])malloc(sizeof(dual[3]) * (size_t)(n * K));
  double sq_lim = sqrt(w->rho_lim), sq_curv = sqrt(w->rho_curv);

  for (int t = 0; t <= H; t++) {
    waypoint* W = &wp[t];
    for (int k = 0; k < nz; k++) W->z[k] = dvar(z[t * nz + k], k);
    dual Rf[CRO_MAX_SEG][9], pf[CRO_MAX_SEG][3];
    fk_chain(rb, W->z, Rf, pf, pts);
    memcpy(W->R, Rf[n - 1], sizeof(W->R));
    memcpy(W->p, pf[n - 1], sizeof(W->p));
    for (int i = 0; i < n; i++)
      for (int j = 0; j < 3; j++) W->u[3 * i + j] = lift_dual(rb, W->z, i, j);

    /* pose objective: IK eq. (8), path following eq. (16) */
    if ((terms & T_TASK) && (pb->kind == CRO_IK || pb->kind == CRO_PATH)) {
      dual rho[3], om[3];
      pose_log(W->R, W->p, pb->task + 12 * t, rho, om);
      for (int c = 0; c < 3; c++) {
        term tm = {t, 1.0, &rho[c]};
        emit_lin(s, w->w_pos, 1, &tm);
      }
      for (int c = 0; c < 3; c++) {
        term tm = {t, 1.0, &om[c]};
        emit_lin(s, w->w_rot, 1, &tm);
      }
    }
    /* actuation bounds, eq. (9): |u_ij| <= u_max_i on the bending part of each tendon */
    for (int i = 0; i < n && (terms & T_LIMITS); i++)
      for (int j = 0; j < 3; j++) {
        dual ub = bend_dual(rb, W->z, i, j);
        term tm = {t, 1.0, &ub};
        emit_hinge(s, sq_lim, rb->u_max[i], 1, &tm);
      }
    /* bending bound, eq. (9): theta_i <= theta_max */
    for (int i = 0; i < n && (terms & T_LIMITS); i++) {
      double th = sqrt(z[t * nz + zc * i] * z[t * nz + zc * i] + z[t * nz + zc * i + 1] * z[t * nz + zc * i + 1]);
      if (th - rb->theta_max > 0.0) {
        dual thd = dsqrt(dadd(dmul(W->z[zc * i], W->z[zc * i]), dmul(W->z[zc * i + 1], W->z[zc * i + 1])));
        term tm = {t, 1.0, &thd};
        emit_hinge(s, sq_curv, rb->theta_max, 1, &tm);
      }
    }
    /* length bounds of extensible segments, eq. (9): L_min_i <= L_i <= L_max_i, one
     * hinge on the distance from the interval's centre beyond its half width */
    for (int i = 0; i < n && zc == 3 && (terms & T_LIMITS); i++) {
      dual off = dshift(seg_len(rb, W->z, i), -0.5 * (rb->L_min[i] + rb->L_max[i]));
      term tm = {t, 1.0, &off};
      emit_hinge(s, sq_lim, 0.5 * (rb->L_max[i] - rb->L_min[i]), 1, &tm);
    }
    /* obstacle clearance and self contact, eq. (10) */
    if (pts && pb->n_sph > 0 && (terms & T_COLL)) collision_rows(rb, w, pb, t, pts, s);
    if (pts && pb->n_poly > 0 && (terms & T_COLL)) polytope_rows(rb, w, pb, t, pts, s);
    if (pts && rb->self_collision && (terms & T_COLL)) self_rows(rb, w, t, pts, s);
  }

  if (pb->kind != CRO_IK && (terms & T_SMOOTH)) {
    double dt = w->dt;
    /* tendon velocity (t >= 1) and acceleration (t >= 2), finite differences (Sec. IV-A) */
    for (int t = 1; t <= H; t++)
      for (int m = 0; m < 3 * n; m++) {
        term tm[2] = {{t, 1.0 / dt, &wp[t].u[m]}, {t - 1, -1.0 / dt, &wp[t - 1].u[m]}};
        emit_lin(s, sqrt(w->w_vel), 2, tm);
        if (is_finite_bound(w->v_max)) emit_hinge(s, sq_lim, w->v_max, 2, tm);
      }
    for (int t = 2; t <= H; t++)
      for (int m = 0; m < 3 * n; m++) {
        double i2 = 1.0 / (dt * dt);
        term tm[3] = {{t, i2, &wp[t].u[m]}, {t - 1, -2.0 * i2, &wp[t - 1].u[m]}, {t - 2, i2, &wp[t - 2].u[m]}};
        emit_lin(s, sqrt(w->w_acc), 3, tm);
        if (is_finite_bound(w->a_max)) emit_hinge(s, sq_lim, w->a_max, 3, tm);
      }
  }
  if (pb->kind == CRO_TRAJ && (terms & T_LEN)) {
    /* tip path length, eq. (11), squared per step */
    for (int t = 1; t <= H; t++)
      for (int c = 0; c < 3; c++) {
        term tm[2] = {{t, 1.0, &wp[t].p[c]}, {t - 1, -1.0, &wp[t - 1].p[c]}};
        emit_lin(s, sqrt(w->w_len), 2, tm);
      }
  }
  if (pb->kind == CRO_TRAJ && (terms & T_ENDS)) {
    /* endpoint equalities q_0 = q_start, q_H = q_goal, penalised (eq. 17) */
    double zs[ND], zg[ND];
    cro_u_to_z(rb, pb->task, zs);
    cro_u_to_z(rb, pb->task + 3 * n, zg);
    for (int k = 0; k < nz; k++) {
      dual e0 = dshift(wp[0].z[k], -zs[k]);
      term t0 = {0, 1.0, &e0};
      emit_lin(s, sqrt(w->rho_eq), 1, &t0);
      dual eH = dshift(wp[H].z[k], -zg[k]);
      term tH = {H, 1.0, &eH};
      emit_lin(s, sqrt(w->rho_eq), 1, &tH);
    }
  }
  free(pts);
  free(wp);
  return s->cost;
}

static double eval_cost(const cro_robot* rb, const cro_weights* w, const cro_problem* pb,
                        const double* z, sink* s) {
  return eval_terms(rb, w, pb, z, s, T_ALL);
}

static sink make_sink(int nz, int N) {
  sink s;
  memset(&s, 0, sizeof(s));
  s.nz = nz;
  s.N = N;
  return s;
}

double cro_cost(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, const double* u,
                double* grad_u) {
  int n = rb->n_seg, zc = cro_ncoord(rb), nz = zc * n, T = pb->H + 1, N = T * nz;
  double* z = (double*)malloc(sizeof(double) * (size_t)N);
  for (int t = 0; t < T; t++) cro_u_to_z(rb, u + 3 * n * t, z + nz * t);
  sink s = make_sink(nz, N);
  double* gz = NULL;
  if (grad_u) {
    gz = (double*)calloc((size_t)N, sizeof(double));
    s.g = gz;
  }
  double c = eval_cost(rb, w, pb, z, &s);
  if (grad_u) {
    /* chain rule through z(u) of cro_u_to_z: da_i/du_ij = -cos(alpha_j)/(1.5 r_i),
     * db_i/du_ij = -sin(alpha_j)/(1.5 r_i), de_i/du_ij = 1/3 */
    for (int t = 0; t < T; t++)
      for (int i = 0; i < n; i++)
        for (int j = 0; j < 3; j++) {
          grad_u[t * 3 * n + 3 * i + j] =
              -(gz[t * nz + zc * i] * cos(alpha_j(j)) + gz[t * nz + zc * i + 1] * sin(alpha_j(j))) /
              (1.5 * rb->r[i]);
          if (zc == 3) grad_u[t * 3 * n + 3 * i + j] += gz[t * nz + zc * i + 2] / 3.0;
        }
    free(gz);
  }
  free(z);
  return c;
}

int cro_residuals(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, const double* z,
                  double* r, double* J, int cap_rows) {
  int nz = cro_ncoord(rb) * rb->n_seg, N = (pb->H + 1) * nz;
  sink s = make_sink(nz, N);
  s.r = r;
  s.J = J;
  s.cap = cap_rows;
  eval_cost(rb, w, pb, z, &s);
  return s.overflow ? -1 : s.rows;
}

/* pose error of one configuration z (eq. 18) with its position and rotation parts */
void cro_pose_error(const cro_robot* rb, const double* z, const double* T, double* out) {
  int n = rb->n_seg;
  nd = 0;
  dual zd[ND], Rf[CRO_MAX_SEG][9], pf[CRO_MAX_SEG][3], rho[3], om[3];
  for (int k = 0; k < cro_ncoord(rb) * n; k++) zd[k] = dcon(z[k]);
  fk_chain(rb, zd, Rf, pf, NULL);
  pose_log(Rf[n - 1], pf[n - 1], T, rho, om);
  double e2 = 0.0;
  for (int c = 0; c < 3; c++) e2 += rho[c].v * rho[c].v + om[c].v * om[c].v;
  double dp2 = 0.0;
  for (int c = 0; c < 3; c++) {
    double d = T[4 * c + 3] - pf[n - 1][c].v;
    dp2 += d * d;
  }
  /* rotation angle of R_ee^T R_t: atan2(|vee(Re - Re^T)|/2, (tr Re - 1)/2) */
  double Re[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++) acc += Rf[n - 1][3 * k + i].v * T[4 * k + j];
      Re[3 * i + j] = acc;
    }
  double vx = 0.5 * (Re[7] - Re[5]), vy = 0.5 * (Re[2] - Re[6]), vz = 0.5 * (Re[3] - Re[1]);
  double cth = 0.5 * (Re[0] + Re[4] + Re[8] - 1.0);
  out[0] = sqrt(e2);
  out[1] = sqrt(dp2);
  out[2] = atan2(sqrt(vx * vx + vy * vy + vz * vz), cth);
}

/* ------------------------------------------------------------------------- */
/* Levenberg-Marquardt (Sec. IV-C) with backtracking line search.              */
/* ------------------------------------------------------------------------- */

int cro_chol_solve(int N, int bw, double* M, double* x) {
  /* factor M = L L^T in place (lower triangle), band |i - j| <= bw */
  for (int j = 0; j < N; j++) {
    int lo = j - bw < 0 ? 0 : j - bw;
    double d = M[(size_t)j * N + j];
    for (int k = lo; k < j; k++) d -= M[(size_t)j * N + k] * M[(size_t)j * N + k];
    if (!(d > 0.0)) return -1;
    double ljj = sqrt(d);
    M[(size_t)j * N + j] = ljj;
    int hi = j + bw >= N ? N - 1 : j + bw;
    for (int i = j + 1; i <= hi; i++) {
      int lo2 = i - bw < 0 ? 0 : i - bw;
      if (lo2 < lo) lo2 = lo;
      double v = M[(size_t)i * N + j];
      for (int k = lo2; k < j; k++) v -= M[(size_t)i * N + k] * M[(size_t)j * N + k];
      M[(size_t)i * N + j] = v / ljj;
    }
  }
  /* forward substitution L y = x */
  for (int i = 0; i < N; i++) {
    int lo = i - bw < 0 ? 0 : i - bw;
    double v = x[i];
    for (int k = lo; k < i; k++) v -= M[(size_t)i * N + k] * x[k];
    x[i] = v / M[(size_t)i * N + i];
  }
  /* back substitution L^T x = y */
  for (int i = N - 1; i >= 0; i--) {
    int hi = i + bw >= N ? N - 1 : i + bw;
    double v = x[i];
    for (int k = i + 1; k <= hi; k++) v -= M[(size_t)k * N + i] * x[k];
    x[i] = v / M[(size_t)i * N + i];
  }
  return 0;
}

/* Half bandwidth of J^T J: a row couples waypoints t-2..t (acceleration). */
static int band_of(const cro_problem* pb, int nz) {
  if (pb->H == 0) return nz - 1;
  if (pb->H == 1) return 2 * nz - 1;
  return 3 * nz - 1;
}

int cro_lm(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, const cro_opts* o,
           double* z, double* lambda, int iters, double* cost_out, int* trials_out) {
  int nz = cro_ncoord(rb) * rb->n_seg, N = (pb->H + 1) * nz, bw = band_of(pb, nz);
  double* Hm = (double*)malloc(sizeof(double) * (size_t)N * N);
  double* g = (double*)malloc(sizeof(double) * (size_t)N);
  double* dlt = (double*)malloc(sizeof(double) * (size_t)N);
  double* zt = (double*)malloc(sizeof(double) * (size_t)N);
  int failed = 0, trials = 0;
  double lam = *lambda;
  double cost0 = NAN;
  for (int it = 0; it < iters; it++) {
    sink s = make_sink(nz, N);
    memset(Hm, 0, sizeof(double) * (size_t)N * N);
    memset(g, 0, sizeof(double) * (size_t)N);
    s.g = g;
    s.Hm = Hm;
    cost0 = eval_cost(rb, w, pb, z, &s);
    if (!isfinite(cost0)) {
      failed = 1;
      break;
    }
    /* (H + lambda D) delta = -g, D = diag(max(H_jj, 1e-12)) (Marquardt scaling) */
    for (int j = 0; j < N; j++) {
      double dj = Hm[(size_t)j * N + j];
      if (dj < 1e-12) dj = 1e-12;
      Hm[(size_t)j * N + j] += lam * dj;
      dlt[j] = -g[j];
    }
    if (cro_chol_solve(N, bw, Hm, dlt) != 0) {
      lam = fmin(10.0 * lam, o->lambda_max);
      continue;
    }
    double gd = 0.0;
    for (int j = 0; j < N; j++) gd += g[j] * dlt[j];
    double alpha = 1.0;
    int accepted = -1;
    for (int tr = 0; tr < o->ls_max; tr++) {
      for (int j = 0; j < N; j++) zt[j] = z[j] + alpha * dlt[j];
      sink sc = make_sink(nz, N);
      double c = eval_cost(rb, w, pb, zt, &sc);
      trials++;
      if (c <= cost0 + 1e-4 * alpha * gd) {
        accepted = tr;
        break;
      }
      alpha *= 0.5;
    }
    if (accepted >= 0) {
      memcpy(z, zt, sizeof(double) * (size_t)N);
      if (accepted == 0) lam = fmax(lam / 10.0, o->lambda_min);
    } else {
      lam = fmin(10.0 * lam, o->lambda_max);
    }
  }
  *lambda = lam;
  if (cost_out) {
    sink s = make_sink(nz, N);
    *cost_out = eval_cost(rb, w, pb, z, &s);
    if (!isfinite(*cost_out)) failed = 1;
  }
  if (trials_out) *trials_out = trials;
  free(zt);
  free(dlt);
  free(g);
  free(Hm);
  return failed;
}

/* ------------------------------------------------------------------------- */
/* SelectTop and the two-stage driver (Algorithm 1).                           */
/* ------------------------------------------------------------------------- */

/* Candidate order: ascending e, ties by index (a stable sort). Failed candidates last. */
static int before(const double* e, const int32_t* failed, int i, int j) {
  int fi = failed ? failed[i] : 0, fj = failed ? failed[j] : 0;
  if (fi != fj) return fj;
  if (e[i] != e[j]) return e[i] < e[j];
  return i < j;
}

void cro_select_top(int S, int nz, const double* z, const double* e, const double* pen,
                    const int32_t* failed, int n_final, double dup_eps, int32_t* idx_out) {
  int* ord = (int*)malloc(sizeof(int) * (size_t)S);
  int* skipped = (int*)calloc((size_t)S, sizeof(int));
  for (int i = 0; i < S; i++) ord[i] = i;
  /* insertion sort: plain and stable */
  for (int i = 1; i < S; i++) {
    int x = ord[i], j = i - 1;
    while (j >= 0 && before(e, failed, x, ord[j])) {
      ord[j + 1] = ord[j];
      j--;
    }
    ord[j + 1] = x;
  }
  int kept = 0;
  for (int q = 0; q < S && kept < n_final; q++) {
    int c = ord[q];
    if (failed && failed[c]) break;
    int dup = -1;
    for (int k = 0; k < kept && dup < 0; k++) {
      double dmax = 0.0;
      for (int m = 0; m < nz; m++) {
        double d = fabs(z[(size_t)c * nz + m] - z[(size_t)idx_out[k] * nz + m]);
        if (d > dmax) dmax = d;
      }
      if (dmax <= dup_eps) dup = k;
    }
    if (dup < 0) {
      idx_out[kept++] = c;
    } else if (pen[c] < pen[idx_out[dup]]) {
      skipped[idx_out[dup]] = 1; /* the replaced one may refill later */
      idx_out[dup] = c;
    } else {
      skipped[c] = 1;
    }
  }
  /* short of n_final: refill from skipped candidates in sorted order */
  for (int q = 0; q < S && kept < n_final; q++) {
    int c = ord[q];
    if (failed && failed[c]) break;
    if (skipped[c]) {
      idx_out[kept++] = c;
      skipped[c] = 0;
    }
  }
  for (int k = kept; k < n_final; k++) idx_out[k] = -1;
  free(skipped);
  free(ord);
}

/* Smallest clearance of configuration u[3n] (eq. 10 with margin 0): over every
 * backbone point and sphere |p - c| - R - r_i and, with self contact, over every
 * pair of points of non-adjacent segments |p - q| - r_i - r_j.  INFINITY when
 * there is nothing to clear. */
static double contact_gap(const cro_robot* rb, const double* sph, int n_sph, const double* u,
                          const cro_problem* poly) {
  int n = rb->n_seg, K = rb->pts_per_seg;
  double gmin = INFINITY;
  int npoly = poly ? poly->n_poly : 0;
  if ((n_sph <= 0 && npoly <= 0 && !rb->self_collision) || K <= 0) return gmin;
  double* P = (double*)malloc(sizeof(double) * 3 * (size_t)(n * K));
  double arc[3 * CRO_MAX_SEG];
  cro_fk(rb, u, arc, NULL, P);
  for (int i = 0; i < n; i++)
    for (int k = 0; k < K; k++)
      for (int m = 0; m < n_sph; m++) {
        const double* S = sph + 4 * m;
        const double* q = P + 3 * (i * K + k);
        double dx = q[0] - S[0], dy = q[1] - S[1], dzz = q[2] - S[2];
        gmin = fmin(gmin, sqrt(dx * dx + dy * dy + dzz * dzz) - S[3] - rb->r[i]);
      }
  /* convex polytopes: signed distance minus the body radius */
  for (int i = 0; i < n; i++)
    for (int k = 0; k < K; k++)
      for (int j = 0; j < npoly; j++) gmin = fmin(gmin, poly_sd(poly, j, P + 3 * (i * K + k), NULL) - rb->r[i]);
  /* self contact between non-adjacent segments */
  for (int i = 0; i < n && rb->self_collision; i++)
    for (int j = i + 2; j < n; j++)
      for (int k = 0; k < K; k++)
        for (int l = 0; l < K; l++) {
          const double* p = P + 3 * (i * K + k);
          const double* q = P + 3 * (j * K + l);
          double dx = q[0] - p[0], dy = q[1] - p[1], dzz = q[2] - p[2];
          gmin = fmin(gmin, sqrt(dx * dx + dy * dy + dzz * dzz) - rb->r[i] - rb->r[j]);
        }
  free(P);
  return gmin;
}

/* Success / status of a solution z (Sec. V-B, with 1 mm / 1 degree thresholds). */
static int32_t assess(const cro_robot* rb, const cro_problem* pb, const double* z, double* err) {
  int n = rb->n_seg, zc = cro_ncoord(rb), nz = zc * n, T = pb->H + 1, K = rb->pts_per_seg;
  double pos = 0.0, rot = 0.0, viol = 0.0, thx = 0.0, gmin = INFINITY;
  int finite = 1;
  for (int t = 0; t < T; t++) {
    const double* zt = z + t * nz;
    for (int k = 0; k < nz; k++)
      if (!isfinite(zt[k])) finite = 0;
    double pe[3];
    if (pb->kind == CRO_IK || pb->kind == CRO_PATH) {
      cro_pose_error(rb, zt, pb->task + 12 * t, pe);
      pos = fmax(pos, pe[1]);
      rot = fmax(rot, pe[2]);
    } else if (t == 0 || t == T - 1) {
      double frames[12 * CRO_MAX_SEG], arc[3 * CRO_MAX_SEG];
      const double* uend = pb->task + (t == 0 ? 0 : 3 * n);
      cro_fk(rb, uend, arc, frames, NULL);
      cro_pose_error(rb, zt, frames + 12 * (n - 1), pe);
      pos = fmax(pos, pe[1]);
      rot = fmax(rot, pe[2]);
    }
    double u[3 * CRO_MAX_SEG];
    cro_z_to_u(rb, zt, u);
    for (int i = 0; i < n; i++) {
      /* tendon bound on the bending part; extensible segments: length within bounds */
      double e = zc == 3 ? zt[zc * i + 2] : 0.0;
      for (int j = 0; j < 3; j++) viol = fmax(viol, fabs(u[3 * i + j] - e) - rb->u_max[i]);
      if (zc == 3) {
        viol = fmax(viol, rb->L_min[i] - (rb->L[i] + e));
        viol = fmax(viol, (rb->L[i] + e) - rb->L_max[i]);
      }
      double th = sqrt(zt[zc * i] * zt[zc * i] + zt[zc * i + 1] * zt[zc * i + 1]);
      thx = fmax(thx, th - rb->theta_max);
    }
    gmin = fmin(gmin, contact_gap(rb, pb->sph, pb->n_sph, u, pb));
  }
  err[0] = pos;
  err[1] = rot;
  if (!finite) return CRO_NONFINITE;
  int32_t st = 0;
  if (viol > 1e-6 || thx > 0.0) st |= CRO_LIMIT_VIOLATION;
  if (gmin < 0.0) st |= CRO_COLLISION;
  if (!(pos <= 1e-3 && rot <= PI / 180.0)) st |= CRO_NOT_CONVERGED;
  if (st == 0) st = CRO_SOLVED;
  return st;
}

/* Success test of one configuration against a pose (Sec. V-B reading): the
 * assessment of a one-waypoint IK problem. */
static int ik_ok(const cro_robot* rb, const cro_problem* pb, const double* T, const double* z) {
  cro_problem one = *pb;
  one.kind = CRO_IK;
  one.H = 0;
  one.task = T;
  double err[2];
  return assess(rb, &one, z, err) == CRO_SOLVED;
}

void cro_path_seeds(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, const cro_opts* o, int S,
                    const double* u_seed, int k, double* z_out) {
  int n = rb->n_seg, nz = cro_ncoord(rb) * n, T = pb->H + 1;
  double* cand = (double*)malloc(sizeof(double) * (size_t)S * T * nz);
  int* ok = (int*)malloc(sizeof(int) * (size_t)S * T);
  int* fin = (int*)malloc(sizeof(int) * (size_t)S * T);
  cro_problem one = *pb;
  one.kind = CRO_IK;
  one.H = 0;
  /* IK at every waypoint from every seed */
  for (int t = 0; t < T; t++) {
    one.task = pb->task + 12 * t;
    for (int s = 0; s < S; s++) {
      double* z = cand + ((size_t)t * S + s) * nz;
      cro_u_to_z(rb, u_seed + ((size_t)s * T + t) * 3 * n, z);
      double lam = o->lambda0;
      int failed = cro_lm(rb, w, &one, o, z, &lam, k, NULL, NULL);
      int finite = 1;
      for (int q = 0; q < nz; q++)
        if (!isfinite(z[q])) finite = 0;
      fin[t * S + s] = finite && !failed;
      ok[t * S + s] = fin[t * S + s] && ik_ok(rb, pb, one.task, z);
    }
  }
  /* assemble one path per seed, nearest neighbour in the infinity norm */
  for (int s = 0; s < S; s++) {
    double* zp = z_out + (size_t)s * T * nz;
    memcpy(zp, cand + (size_t)s * nz, sizeof(double) * nz);
    for (int t = 1; t < T; t++) {
      const double* prev = zp + (size_t)(t - 1) * nz;
      int best = -1;
      double bd = 0.0;
      for (int pass = 0; pass < 2 && best < 0; pass++) {
        for (int j = 0; j < S; j++) {
          if (pass == 0 ? !ok[t * S + j] : !fin[t * S + j]) continue;
          const double* zj = cand + ((size_t)t * S + j) * nz;
          double d = 0.0;
          for (int q = 0; q < nz; q++) d = fmax(d, fabs(zj[q] - prev[q]));
          if (best < 0 || d < bd) {
            best = j;
            bd = d;
          }
        }
      }
      const double* src = best >= 0 ? cand + ((size_t)t * S + best) * nz : prev;
      memcpy(zp + (size_t)t * nz, src, sizeof(double) * nz);
    }
  }
  free(fin);
  free(ok);
  free(cand);
}

int cro_solve(const cro_robot* rb, const cro_weights* w, const cro_problem* pb, const cro_opts* o, int S,
              const double* u_seed, double* u_out, double* err_out, int32_t* status, int32_t* best_idx,
              double* best_cost) {
  int n = rb->n_seg, nz = cro_ncoord(rb) * n, T = pb->H + 1, N = T * nz;
  if (n < 1 || n > CRO_MAX_SEG || S < 1 || pb->H < 0 || (pb->kind == CRO_IK && pb->H != 0) ||
      (pb->kind == CRO_TRAJ && pb->H < 1))
    return -1;
  double* z = (double*)malloc(sizeof(double) * (size_t)S * N);
  double* lam = (double*)malloc(sizeof(double) * (size_t)S);
  double* cost = (double*)malloc(sizeof(double) * (size_t)S);
  int32_t* failed = (int32_t*)malloc(sizeof(int32_t) * (size_t)S);

  /* stage 1: ParallelOptimize over every seed for k_init iterations */
  if (pb->kind == CRO_PATH && o->k_seed > 0) cro_path_seeds(rb, w, pb, o, S, u_seed, o->k_seed, z);
  for (int s = 0; s < S; s++) {
    if (!(pb->kind == CRO_PATH && o->k_seed > 0))
      for (int t = 0; t < T; t++) cro_u_to_z(rb, u_seed + (size_t)s * T * 3 * n + 3 * n * t, z + (size_t)s * N + nz * t);
    lam[s] = o->lambda0;
    failed[s] = cro_lm(rb, w, pb, o, z + (size_t)s * N, &lam[s], o->k_init, &cost[s], NULL);
  }

  int ncand = S;
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S > o->n_final ? S : o->n_final));
  for (int s = 0; s < S; s++) cand[s] = s;
  if (o->n_final > 0) {
    /* SelectTop: rank by the unweighted pose error (eq. 8) for IK, by the total
     * cost for path/trajectory; near-duplicate ties go to the lower collision penalty */
    double* e = (double*)malloc(sizeof(double) * (size_t)S);
    double* pen = (double*)malloc(sizeof(double) * (size_t)S);
    for (int s = 0; s < S; s++) {
      if (pb->kind == CRO_IK) {
        double pe[3];
        cro_pose_error(rb, z + (size_t)s * N, pb->task, pe);
        e[s] = pe[0];
      } else {
        e[s] = cost[s];
      }
      if (!isfinite(e[s])) failed[s] = 1;
      /* collision part of the cost alone (the tie-break of SelectTop) */
      sink sc = make_sink(nz, N);
      double c = eval_terms(rb, w, pb, z + (size_t)s * N, &sc, T_COLL);
      pen[s] = c;
    }
    ncand = o->n_final;
    cro_select_top(S, N, z, e, pen, failed, o->n_final, o->dup_eps, cand);
    free(pen);
    free(e);
    /* stage 2: refine the kept candidates from a fresh lambda */
    for (int k = 0; k < ncand; k++) {
      int s = cand[k];
      if (s < 0) continue;
      lam[s] = o->lambda0;
      failed[s] = cro_lm(rb, w, pb, o, z + (size_t)s * N, &lam[s], o->k_final, &cost[s], NULL);
    }
  }

  /* q* = argmin of the final cost, ties to the lowest seed index */
  int best = -1;
  for (int k = 0; k < ncand; k++) {
    int s = cand[k];
    if (s < 0 || failed[s] || !isfinite(cost[s])) continue;
    if (best < 0 || cost[s] < cost[best] || (cost[s] == cost[best] && s < best)) best = s;
  }
  int rc = 0;
  if (best < 0) {
    for (int q = 0; q < N / nz * 3 * n; q++) u_out[q] = NAN;
    err_out[0] = err_out[1] = NAN;
    *status = CRO_NONFINITE;
    *best_idx = -1;
    *best_cost = NAN;
  } else {
    for (int t = 0; t < T; t++) cro_z_to_u(rb, z + (size_t)best * N + nz * t, u_out + 3 * n * t);
    *status = assess(rb, pb, z + (size_t)best * N, err_out);
    *best_idx = best;
    *best_cost = cost[best];
  }
  free(cand);
  free(failed);
  free(cost);
  free(lam);
  free(z);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* SampleSeeds (Algorithm 1; Sec. IV-B: seeds inside the bounds, seeds that    */
/* collide at once are drawn again).                                          */
/* ------------------------------------------------------------------------- */

/* Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds; each multiplies words 0 and 2 by the
 * round multipliers into 128-bit products and mixes the high halves with the
 * other words and the key, the key advancing by the two Weyl increments
 * between rounds. */
void cro_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    unsigned __int128 p0 = (unsigned __int128)M0 * c0, p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0, hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* uniform j of the stream of (problem p, seed s, attempt a): word j mod 4 of
 * Philox4x64-10 at counter (j div 4, a, s, p), its top 53 bits scaled to [0, 1) */
static double seed_uniform(const uint64_t key[2], int64_t p, int32_t s, int32_t a, int64_t j) {
  uint64_t ctr[4] = {(uint64_t)(j >> 2), (uint64_t)a, (uint64_t)s, (uint64_t)p}, out[4];
  cro_philox4x64(ctr, key, out);
  return (double)(out[j & 3] >> 11) * 0x1.0p-53;
}

double cro_contact_gap(const cro_robot* rb, const double* sph, int n_sph, const double* u) {
  return contact_gap(rb, sph, n_sph, u, NULL);
}

int32_t cro_sample_seed(const cro_robot* rb, const double* sph, int n_sph, const uint64_t key[2], int64_t p,
                        int32_t s, int32_t max_attempts, double* u) {
  int n = rb->n_seg;
  int32_t a = 0;
  for (;; a++) {
    int64_t j = 0;
    for (int i = 0; i < n; i++) {
      const double b = rb->u_max[i];
      double ub[3] = {0.0, 0.0, 0.0}, worst = 0.0;
      int ok = 0;
      for (int tries = 0; tries < CRO_SEED_TRIPLES && !ok; tries++) {
        double x[3];
        for (int k = 0; k < 3; k++) x[k] = b * (2.0 * seed_uniform(key, p, s, a, j++) - 1.0);
        const double mean = (x[0] + x[1] + x[2]) / 3.0;
        worst = 0.0;
        for (int k = 0; k < 3; k++) {
          ub[k] = x[k] - mean;
          worst = fmax(worst, fabs(ub[k]));
        }
        /* bending angle of the zero-sum part: |(a, b)| of eq. (4) inverted */
        double pc = 0.0, ps = 0.0;
        for (int k = 0; k < 3; k++) {
          pc += ub[k] * cos(alpha_j(k));
          ps += ub[k] * sin(alpha_j(k));
        }
        const double th = sqrt(pc * pc + ps * ps) / (1.5 * rb->r[i]);
        ok = worst <= b && th <= rb->theta_max;
      }
      if (!ok) {
        /* no triple inside the bounds: the last one scaled onto them */
        double pc = 0.0, ps = 0.0;
        for (int k = 0; k < 3; k++) {
          pc += ub[k] * cos(alpha_j(k));
          ps += ub[k] * sin(alpha_j(k));
        }
        const double th = sqrt(pc * pc + ps * ps) / (1.5 * rb->r[i]);
        double f = fmin(worst > 0.0 ? b / worst : 1.0, th > 0.0 ? rb->theta_max / th : 1.0);
        for (int k = 0; k < 3; k++) ub[k] *= f;
      }
      /* extensible: the extension drawn within the length bounds of eq. (9) */
      double e = 0.0;
      if (rb->extensible)
        e = (rb->L_min[i] - rb->L[i]) + (rb->L_max[i] - rb->L_min[i]) * seed_uniform(key, p, s, a, j++);
      for (int k = 0; k < 3; k++) u[3 * i + k] = ub[k] + e;
    }
    if (a + 1 >= max_attempts || !(contact_gap(rb, sph, n_sph, u, NULL) < 0.0)) break;
  }
  return contact_gap(rb, sph, n_sph, u, NULL) < 0.0 ? -(a + 1) : a + 1;
}
