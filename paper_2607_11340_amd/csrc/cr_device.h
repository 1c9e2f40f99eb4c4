// cr_device.h -- device-side kinematics, cost and Levenberg-Marquardt pieces for
// gfx950.  Everything is templated on the arithmetic type T (float or double) and,
// where the segment count sizes register arrays, on NS (1..6) so that per-seed
// state lives in VGPRs with compile-time indexing.
//
// Coordinates: each segment i is described by its bending coordinates
// (a_i, b_i) = theta_i (cos phi_i, sin phi_i) (Sec. III-A, q = (theta, phi, L) with
// L fixed); tendon displacements u map to them linearly through eq. (4).  Robots
// with extensible segments (the extendable robots of Sec. V-B) carry a third
// coordinate per segment, the extension e_i = mean_j u_ij, with L_i = L[i] + e_i;
// the functions of the generic per-configuration path take EXT for them (NC = 3
// coordinates per segment, stored a, b, e).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cr_solver.h"

// Device functions are also compiled for the host so that the same arithmetic
// can be replayed with an op-counting scalar (algorithmic flop accounting).
#define CR_HD __host__ __device__ __forceinline__

namespace crk {

// ---------------------------------------------------------------------------
// Parameters in the kernel's arithmetic type (passed by value as kernel args).
// ---------------------------------------------------------------------------

template <typename T>
struct RobotT {
  int n, K;
  T L[CR_MAX_SEG], r[CR_MAX_SEG], umax[CR_MAX_SEG];
  T theta_max;
  // FP64 copies of the geometry for the FP64 chains (stage 2, assessment)
  double Ld[CR_MAX_SEG], rd[CR_MAX_SEG], umaxd[CR_MAX_SEG], theta_maxd;
  // extensible segments: centre and half width of each length interval (eq. 9)
  int ext;
  int self;  // 1: contact between non-adjacent segments counts as collision (eq. 10)
  T Lmid[CR_MAX_SEG], Lhalf[CR_MAX_SEG];
  double Lmidd[CR_MAX_SEG], Lhalfd[CR_MAX_SEG];
};

template <typename T>
struct WeightsT {
  T w_pos, w_rot;      // pose residual weights
  T sq_lim, sq_curv;   // square roots of the bound penalties (residual scales)
  T sq_coll, margin;
  T sq_eq, sq_len, sq_vel, sq_acc;
  T v_max, a_max, dt;
  int has_vmax, has_amax;
  double margind;  // FP64 copy for the clearance hinge
};

// ---------------------------------------------------------------------------
// Small helpers.
// ---------------------------------------------------------------------------

template <typename T>
CR_HD T tsqrt(T x);
template <>
CR_HD float tsqrt<float>(float x) { return sqrtf(x); }
template <>
CR_HD double tsqrt<double>(double x) { return sqrt(x); }

template <typename T>
CR_HD T tatan2(T y, T x);
template <>
CR_HD float tatan2<float>(float y, float x) { return atan2f(y, x); }
template <>
CR_HD double tatan2<double>(double y, double x) { return atan2(y, x); }

template <typename T>
CR_HD void tsincos(T x, T* s, T* c);
template <>
CR_HD void tsincos<float>(float x, float* s, float* c) { sincosf(x, s, c); }
template <>
CR_HD void tsincos<double>(double x, double* s, double* c) { sincos(x, s, c); }

// 1/x: the hardware reciprocal (1 ulp) in FP32, an IEEE division in FP64.
template <typename T>
CR_HD T trcp(T x) {
  return T(1) / x;
}
template <>
CR_HD float trcp<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

template <typename T>
CR_HD bool tfinite(T x) {
  return __builtin_isfinite(x);
}

template <typename T>
CR_HD void cross3(const T* a, const T* b, T* c) {
  T c0 = a[1] * b[2] - a[2] * b[1];
  T c1 = a[2] * b[0] - a[0] * b[2];
  T c2 = a[0] * b[1] - a[1] * b[0];
  c[0] = c0;
  c[1] = c1;
  c[2] = c2;
}
template <typename T>
CR_HD T dot3(const T* a, const T* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
// y = M x  (row-major 3x3)
template <typename T>
CR_HD void mv3(const T* M, const T* x, T* y) {
  T y0 = M[0] * x[0] + M[1] * x[1] + M[2] * x[2];
  T y1 = M[3] * x[0] + M[4] * x[1] + M[5] * x[2];
  T y2 = M[6] * x[0] + M[7] * x[1] + M[8] * x[2];
  y[0] = y0;
  y[1] = y1;
  y[2] = y2;
}
// y = M^T x
template <typename T>
CR_HD void mtv3(const T* M, const T* x, T* y) {
  T y0 = M[0] * x[0] + M[3] * x[1] + M[6] * x[2];
  T y1 = M[1] * x[0] + M[4] * x[1] + M[7] * x[2];
  T y2 = M[2] * x[0] + M[5] * x[1] + M[8] * x[2];
  y[0] = y0;
  y[1] = y1;
  y[2] = y2;
}
// C = A B
template <typename T>
CR_HD void mm3(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// ---------------------------------------------------------------------------
// Power series in s = theta^2.  (-1)^k / (2k + OFF)!  evaluated by Horner.
// ---------------------------------------------------------------------------

constexpr double inv_factorial(int m) {
  double f = 1.0;
  for (int i = 2; i <= m; ++i) f *= (double)i;
  return 1.0 / f;
}
constexpr double alt_coef(int k, int off) { return ((k & 1) ? -1.0 : 1.0) * inv_factorial(2 * k + off); }

// sum_{k<NT} alt_coef(k, OFF) s^k
template <typename T, int OFF, int NT>
CR_HD T alt_series(T s) {
  T acc = T(alt_coef(NT - 1, OFF));
#pragma unroll
  for (int k = NT - 2; k >= 0; --k) acc = acc * s + T(alt_coef(k, OFF));
  return acc;
}
// d/ds of the above
template <typename T, int OFF, int NT>
CR_HD T alt_series_d(T s) {
  T acc = T((NT - 1) * alt_coef(NT - 1, OFF));
#pragma unroll
  for (int k = NT - 2; k >= 1; --k) acc = acc * s + T(k * alt_coef(k, OFF));
  return acc;
}

template <typename T>
struct Prec;
// Series lengths and switch points.  FP32 keeps the polynomial up to s = 4
// (theta < 2 rad, every bend the bounded robots reach), so the common path has
// no transcendental call; the largest term there is 2/3 of the leading one, so
// the sum loses no more than an ulp.
template <>
struct Prec<float> {
  static constexpr int NT = 11;          // series terms for s < s_switch
  static constexpr float s_switch = 4.0f;
  static constexpr int NG = 8;           // gamma series terms for q < g_switch
  static constexpr float g_switch = 4.0f;
};
template <>
struct Prec<double> {
  static constexpr int NT = 10;
  static constexpr double s_switch = 1.0;
  static constexpr int NG = 8;
  static constexpr double g_switch = 0.25;
};

// Arc coefficients of Rodrigues' formula for the in-plane rotation vector
// w = (-b, a, 0), |w| = theta, s = theta^2:
//   A = (1 - cos theta)/s,  B = sin(theta)/theta,  C = (theta - sin theta)/theta^3
// and the s-derivatives A', B'.  Series below s = 1 (no cancellation), closed
// forms above.
template <typename T>
struct ArcCoef {
  T A, B, C, Ap, Bp;
};

template <typename T, bool DERIV>
CR_HD ArcCoef<T> arc_coef(T s) {
  constexpr int NT = Prec<T>::NT;
  ArcCoef<T> c;
  if (s < T(Prec<T>::s_switch)) {
    c.A = alt_series<T, 2, NT>(s);
    c.B = alt_series<T, 1, NT>(s);
    if (DERIV) {
      c.C = alt_series<T, 3, NT>(s);
      c.Ap = alt_series_d<T, 2, NT>(s);
      c.Bp = alt_series_d<T, 1, NT>(s);
    }
  } else {
    T th = tsqrt(s), sh, ch;
    tsincos(T(0.5) * th, &sh, &ch);
    T inv_s = trcp(s);
    c.A = T(2) * sh * sh * inv_s;
    c.B = T(2) * sh * ch * trcp(th);
    if (DERIV) {
      T cth = ch * ch - sh * sh;
      c.C = (T(1) - c.B) * inv_s;
      c.Ap = (T(0.5) * c.B - c.A) * inv_s;
      c.Bp = T(0.5) * (cth - c.B) * inv_s;
    }
  }
  return c;
}

// gamma(q) = (1 - (theta/2) cot(theta/2)) / q and dgamma/dq, q = theta^2: the
// [w]_x^2 coefficient of the inverse left Jacobian V^-1 = I - [w]_x/2 + gamma [w]_x^2.
// Series: gamma = sum_{k>=1} |B_2k| q^(k-1) / (2k)! (Bernoulli numbers).
CR_HD constexpr double bern_gamma_coef(int k) {
  // |B_2k| / (2k)!, k = 1..9
  return k == 1   ? (1.0 / 6.0) * inv_factorial(2)
         : k == 2 ? (1.0 / 30.0) * inv_factorial(4)
         : k == 3 ? (1.0 / 42.0) * inv_factorial(6)
         : k == 4 ? (1.0 / 30.0) * inv_factorial(8)
         : k == 5 ? (5.0 / 66.0) * inv_factorial(10)
         : k == 6 ? (691.0 / 2730.0) * inv_factorial(12)
         : k == 7 ? (7.0 / 6.0) * inv_factorial(14)
         : k == 8 ? (3617.0 / 510.0) * inv_factorial(16)
                  : (43867.0 / 798.0) * inv_factorial(18);
}

template <typename T, bool DERIV>
CR_HD void gamma_coef(T q, T* gam, T* dgam) {
  constexpr int NG = Prec<T>::NG;
  if (q < T(Prec<T>::g_switch)) {
    T acc = T(bern_gamma_coef(NG));
#pragma unroll
    for (int k = NG - 1; k >= 1; --k) acc = acc * q + T(bern_gamma_coef(k));
    *gam = acc;
    if (DERIV) {
      T d = T((NG - 1) * bern_gamma_coef(NG));
#pragma unroll
      for (int k = NG - 1; k >= 2; --k) d = d * q + T((k - 1) * bern_gamma_coef(k));
      *dgam = d;
    }
  } else {
    T th = tsqrt(q), sh, ch;
    tsincos(T(0.5) * th, &sh, &ch);
    const T ish = trcp(sh), iq = trcp(q);
    T cot = ch * ish;
    T h = T(0.5) * th * cot;
    T g = (T(1) - h) * iq;
    *gam = g;
    if (DERIV) {
      T dh = T(0.5) * cot - T(0.25) * th * ish * ish;
      *dgam = (-dh * T(0.5) * trcp(th) - g) * iq;
    }
  }
}

// ---------------------------------------------------------------------------
// Tendon map (eq. 4) for three tendons at 0, 120, 240 degrees:
//   u_j = -r (a cos alpha_j + b sin alpha_j)
//   a = (u_2 + u_3 - 2 u_1) / (3 r),  b = (u_3 - u_2) / (sqrt(3) r)
// ---------------------------------------------------------------------------

template <typename T>
CR_HD void u_to_ab(T u0, T u1, T u2, T r, T* a, T* b) {
  const T ir = trcp(r);
  *a = (u1 + u2 - T(2) * u0) * (T(1.0 / 3.0) * ir);
  *b = (u2 - u1) * (T(0.57735026918962576451) * ir);
}

template <typename T>
CR_HD void ab_to_u(T a, T b, T r, T* u) {
  const T h3 = T(0.86602540378443864676);  // sqrt(3)/2
  u[0] = -r * a;
  u[1] = r * (T(0.5) * a - h3 * b);
  u[2] = r * (T(0.5) * a + h3 * b);
}

// d u_j / d(a, b)
template <typename T>
CR_HD void lift_row(int j, T r, T* da, T* db) {
  const T h3 = T(0.86602540378443864676);
  *da = j == 0 ? -r : T(0.5) * r;
  *db = j == 0 ? T(0) : (j == 1 ? -h3 * r : h3 * r);
}

// ---------------------------------------------------------------------------
// Segment transform (eq. 1-3):  R = I + B [w]_x + A [w]_x^2,  w = (-b, a, 0),
// d = L (A a, A b, B).
// ---------------------------------------------------------------------------

template <typename T>
CR_HD void seg_R_d(T a, T b, T L, const ArcCoef<T>& c, T* R, T* d) {
  T s = a * a + b * b;
  T Aab = c.A * a * b;
  R[0] = T(1) - c.A * a * a;
  R[1] = -Aab;
  R[2] = c.B * a;
  R[3] = -Aab;
  R[4] = T(1) - c.A * b * b;
  R[5] = c.B * b;
  R[6] = -c.B * a;
  R[7] = -c.B * b;
  R[8] = T(1) - c.A * s;
  d[0] = L * c.A * a;
  d[1] = L * c.A * b;
  d[2] = L * c.B;
}

// Length of segment i at coordinates z (NC per segment).
template <bool EXT, typename T>
CR_HD T seg_len(const RobotT<T>& rb, const T* z, int i) {
  if constexpr (EXT) return rb.L[i] + z[3 * i + 2];
  else return rb.L[i];
}

// Value-only chain of NS segments: tip rotation Rc and position pc.
template <int NS, typename T, bool EXT = false>
CR_HD void fk_tip(const RobotT<T>& rb, const T* z, T* Rc, T* pc) {
  constexpr int NC = EXT ? 3 : 2;
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = (k % 4 == 0) ? T(1) : T(0);
  pc[0] = pc[1] = pc[2] = T(0);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    T a = z[NC * i], b = z[NC * i + 1];
    ArcCoef<T> c = arc_coef<T, false>(a * a + b * b);
    T Ri[9], di[3], q[3], Rn[9];
    seg_R_d(a, b, seg_len<EXT>(rb, z, i), c, Ri, di);
    mv3(Rc, di, q);
    pc[0] += q[0];
    pc[1] += q[1];
    pc[2] += q[2];
    mm3(Rc, Ri, Rn);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = Rn[k];
  }
}

// ---------------------------------------------------------------------------
// SE(3) logarithm of E = [Re | te] (eq. 8, 16, 18):
//   w = Log_SO3(Re), rho = V^-1(w) te.
// ---------------------------------------------------------------------------

template <typename T, bool DERIV>
CR_HD void log_se3(const T* Re, const T* te, T* w, T* rho, T* gam, T* dgam) {
  T c = T(0.5) * (Re[0] + Re[4] + Re[8] - T(1));
  T v[3] = {T(0.5) * (Re[7] - Re[5]), T(0.5) * (Re[2] - Re[6]), T(0.5) * (Re[3] - Re[1])};
  T x = dot3(v, v);  // sin^2(theta)
  if (c > T(-0.9)) {
    T f;
    if (c > T(0) && x < T(1e-8)) {
      f = T(1) + x * (T(1.0 / 6.0) + x * T(3.0 / 40.0));  // theta / sin(theta)
    } else {
      T sn = tsqrt(x);
      f = tatan2(sn, c) * trcp(sn);
    }
    w[0] = f * v[0];
    w[1] = f * v[1];
    w[2] = f * v[2];
  } else {
    // near pi: (Re + Re^T)/2 = c I + (1 - c) n n^T; axis from the largest diagonal
    T inv = trcp(T(1) - c);
    T d0 = (Re[0] - c) * inv, d1 = (Re[4] - c) * inv, d2 = (Re[8] - c) * inv;
    T n[3];
    if (d0 >= d1 && d0 >= d2) {
      T s = tsqrt(d0), is = T(0.5) * inv * trcp(s);
      n[0] = s;
      n[1] = (Re[1] + Re[3]) * is;
      n[2] = (Re[2] + Re[6]) * is;
    } else if (d1 >= d2) {
      T s = tsqrt(d1), is = T(0.5) * inv * trcp(s);
      n[0] = (Re[1] + Re[3]) * is;
      n[1] = s;
      n[2] = (Re[5] + Re[7]) * is;
    } else {
      T s = tsqrt(d2), is = T(0.5) * inv * trcp(s);
      n[0] = (Re[2] + Re[6]) * is;
      n[1] = (Re[5] + Re[7]) * is;
      n[2] = s;
    }
    T sn = dot3(n, v);
    bool flip = sn < T(0);
    if (sn == T(0)) flip = (n[0] != T(0)) ? (n[0] < T(0)) : ((n[1] != T(0)) ? (n[1] < T(0)) : (n[2] < T(0)));
    if (flip) {
      n[0] = -n[0];
      n[1] = -n[1];
      n[2] = -n[2];
      sn = -sn;
    }
    T th = tatan2(sn, c);
    w[0] = th * n[0];
    w[1] = th * n[1];
    w[2] = th * n[2];
  }
  T g, dg = T(0);
  gamma_coef<T, DERIV>(dot3(w, w), &g, &dg);
  T u1[3], u2[3];
  cross3(w, te, u1);
  cross3(w, u1, u2);
  rho[0] = te[0] - T(0.5) * u1[0] + g * u2[0];
  rho[1] = te[1] - T(0.5) * u1[1] + g * u2[1];
  rho[2] = te[2] - T(0.5) * u1[2] + g * u2[2];
  *gam = g;
  if (DERIV) *dgam = dg;
}

// Re = R^T Rt, te = R^T (pt - p) for a target pose T[12] (3x4 row-major).
template <typename T>
CR_HD void relative_pose(const T* R, const T* p, const T* Tt, T* Re, T* te) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Re[3 * i + j] = R[i] * Tt[j] + R[3 + i] * Tt[4 + j] + R[6 + i] * Tt[8 + j];
  T dp[3] = {Tt[3] - p[0], Tt[7] - p[1], Tt[11] - p[2]};
  mtv3(R, dp, te);
}

// ---------------------------------------------------------------------------
// Bound penalties shared by every task (eq. 9): tendon hinge and bending hinge.
// ---------------------------------------------------------------------------

// One segment's bound residuals from its bending coordinates (eq. 9):
// tendon hinges sq_lim max(0, |u_j| - u_max) and the bending hinge
// sq_curv max(0, theta - theta_max).  ru[j] / rth are 0 when inactive.
// TH is the type the violations are formed in (the kernel's chain type).
template <typename TH, typename T>
CR_HD void bound_residuals(const RobotT<T>& rb, const WeightsT<T>& w, int i, TH a, TH b, TH* ru, TH* sgn, TH* rth) {
  const TH r = sizeof(TH) == 8 ? (TH)rb.rd[i] : (TH)rb.r[i];
  const TH umax = sizeof(TH) == 8 ? (TH)rb.umaxd[i] : (TH)rb.umax[i];
  const TH thmax = sizeof(TH) == 8 ? (TH)rb.theta_maxd : (TH)rb.theta_max;
  TH u[3];
  ab_to_u(a, b, r, u);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const TH viol = fabs(u[j]) - umax;
    ru[j] = viol > TH(0) ? (TH)w.sq_lim * viol : TH(0);
    sgn[j] = u[j] < TH(0) ? TH(-1) : TH(1);
  }
  const TH s = a * a + b * b;
  // theta > theta_max  <=>  theta^2 > theta_max^2: the square root is taken only when active
  *rth = s > thmax * thmax ? (TH)w.sq_curv * (tsqrt(s) - thmax) : TH(0);
}

// Length hinge of an extensible segment (eq. 9, L_min <= L_i <= L_max):
// sq_lim max(0, |L_i - mid| - half) with L_i = L[i] + e; *sgn = sign(L_i - mid).
template <typename TH, typename T>
CR_HD TH length_residual(const RobotT<T>& rb, const WeightsT<T>& w, int i, TH e, TH* sgn) {
  const TH L0 = sizeof(TH) == 8 ? (TH)rb.Ld[i] : (TH)rb.L[i];
  const TH mid = sizeof(TH) == 8 ? (TH)rb.Lmidd[i] : (TH)rb.Lmid[i];
  const TH half = sizeof(TH) == 8 ? (TH)rb.Lhalfd[i] : (TH)rb.Lhalf[i];
  const TH off = (L0 + e) - mid;
  *sgn = off < TH(0) ? TH(-1) : TH(1);
  const TH viol = fabs(off) - half;
  return viol > TH(0) ? (TH)w.sq_lim * viol : TH(0);
}

template <int NS, typename T, bool EXT = false>
CR_HD T bounds_cost(const RobotT<T>& rb, const WeightsT<T>& w, const T* z) {
  constexpr int NC = EXT ? 3 : 2;
  T c = T(0);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    T ru[3], sg[3], rth;
    bound_residuals<T>(rb, w, i, z[NC * i], z[NC * i + 1], ru, sg, &rth);
    c += T(0.5) * (ru[0] * ru[0] + ru[1] * ru[1] + ru[2] * ru[2] + rth * rth);
    if constexpr (EXT) {
      T se;
      const T rl = length_residual<T>(rb, w, i, z[NC * i + 2], &se);
      c += T(0.5) * rl * rl;
    }
  }
  return c;
}

// packed lower-triangular index
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Adds the bound rows to cost, g = J^T r and H = J^T J (packed lower) for one configuration.
// `off` is the column offset of this configuration's (a, b) block.
template <int NS, int NZT, typename T, bool EXT = false>
CR_HD void bounds_normal_eq(const RobotT<T>& rb, const WeightsT<T>& w, const T* z, int off, T* Hp, T* g, T& cost) {
  constexpr int NC = EXT ? 3 : 2;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const T a = z[NC * i], b = z[NC * i + 1];
    T ru[3], sg[3], rth;
    bound_residuals<T>(rb, w, i, a, b, ru, sg, &rth);
    const int ca = off + NC * i, cb = off + NC * i + 1;
    if constexpr (EXT) {
      T se;
      const T rl = length_residual<T>(rb, w, i, z[NC * i + 2], &se);
      if (rl > T(0)) {
        const int ce = off + NC * i + 2;
        const T je = se * w.sq_lim;
        cost += T(0.5) * rl * rl;
        g[ce] += je * rl;
        Hp[tri(ce, ce)] += je * je;
      }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (ru[j] > T(0)) {
        T ja, jb;
        lift_row(j, rb.r[i], &ja, &jb);
        ja *= sg[j] * w.sq_lim;
        jb *= sg[j] * w.sq_lim;
        cost += T(0.5) * ru[j] * ru[j];
        g[ca] += ja * ru[j];
        g[cb] += jb * ru[j];
        Hp[tri(ca, ca)] += ja * ja;
        Hp[tri(cb, ca)] += jb * ja;
        Hp[tri(cb, cb)] += jb * jb;
      }
    }
    if (rth > T(0)) {
      const T ith = trcp(tsqrt(a * a + b * b));
      const T ja = w.sq_curv * a * ith, jb = w.sq_curv * b * ith;
      cost += T(0.5) * rth * rth;
      g[ca] += ja * rth;
      g[cb] += jb * rth;
      Hp[tri(ca, ca)] += ja * ja;
      Hp[tri(cb, ca)] += jb * ja;
      Hp[tri(cb, cb)] += jb * jb;
    }
  }
}

// ---------------------------------------------------------------------------
// IK cost (value) and Gauss-Newton normal equations for one configuration.
// ---------------------------------------------------------------------------

// Pose part: returns 1/2 |(w_pos rho, w_rot w)|^2; optionally the unweighted |log|.
template <int NS, typename T, bool EXT = false>
CR_HD T ik_cost(const RobotT<T>& rb, const WeightsT<T>& w, const T* Tt, const T* z,
                                     T* e_out) {
  T Rc[9], pc[3], Re[9], te[3], om[3], rho[3], gam, dg;
  fk_tip<NS, T, EXT>(rb, z, Rc, pc);
  relative_pose(Rc, pc, Tt, Re, te);
  log_se3<T, false>(Re, te, om, rho, &gam, &dg);
  T r2 = w.w_pos * w.w_pos * dot3(rho, rho) + w.w_rot * w.w_rot * dot3(om, om);
  if (e_out) *e_out = tsqrt(dot3(rho, rho) + dot3(om, om));
  return T(0.5) * r2 + bounds_cost<NS, T, EXT>(rb, w, z);
}

// Normal equations H = J^T J (packed lower, 2NS x 2NS), g = J^T r and cost at z.
//
// Pose Jacobian: a change of z_k moves the tip by the spatial twist
// (W_k, dp_k) with W_k = R_{0,i-1} J_l(w_i) e_k' and dp_k = R_{0,i-1} dd_i/dz_k
// + W_k x (p_ee - p_{0,i}); in the tip frame that is (Jv, Jw) = R_ee^T (dp, W).
// With E = T_ee^-1 T_t and E -> exp(-xi) E, the log changes by
//   dw = -V^-1 Jw,  drho = -V^-1 (Jv - t x Jw) - N V^-1 Jw,
//   N y = y x... = t x y / 2 + 2 gamma' (w . y) (w x (w x t)) - gamma (w x t) x y - gamma w x (t x y).
template <int NS, typename T>
CR_HD T ik_normal_eq(const RobotT<T>& rb, const WeightsT<T>& w, const T* Tt, const T* z,
                                          T* Hp, T* g) {
  constexpr int NZ = 2 * NS;
  T Rc[9], pc[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = (k % 4 == 0) ? T(1) : T(0);
  pc[0] = pc[1] = pc[2] = T(0);
  T Wc[NZ][3], Pc[NZ][3], Pi[NS][3];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    T a = z[2 * i], b = z[2 * i + 1];
    ArcCoef<T> c = arc_coef<T, true>(a * a + b * b);
    T Ri[9], di[3];
    seg_R_d(a, b, rb.L[i], c, Ri, di);
    const T L = rb.L[i];
    // rotation-vector derivatives pushed to the parent frame: R_i J_r = J_l
    T wa[3] = {-c.C * a * b, T(1) - c.C * b * b, -c.A * b};
    T wb[3] = {c.C * a * a - T(1), c.C * a * b, c.A * a};
    T dda[3] = {L * (c.A + T(2) * a * a * c.Ap), L * T(2) * a * b * c.Ap, L * T(2) * a * c.Bp};
    T ddb[3] = {L * T(2) * a * b * c.Ap, L * (c.A + T(2) * b * b * c.Ap), L * T(2) * b * c.Bp};
    mv3(Rc, wa, Wc[2 * i]);
    mv3(Rc, wb, Wc[2 * i + 1]);
    mv3(Rc, dda, Pc[2 * i]);
    mv3(Rc, ddb, Pc[2 * i + 1]);
    T q[3], Rn[9];
    mv3(Rc, di, q);
    pc[0] += q[0];
    pc[1] += q[1];
    pc[2] += q[2];
    mm3(Rc, Ri, Rn);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = Rn[k];
    Pi[i][0] = pc[0];
    Pi[i][1] = pc[1];
    Pi[i][2] = pc[2];
  }
  T Re[9], te[3], om[3], rho[3], gam, dgam;
  relative_pose(Rc, pc, Tt, Re, te);
  log_se3<T, true>(Re, te, om, rho, &gam, &dgam);
  T r[6] = {w.w_pos * rho[0], w.w_pos * rho[1], w.w_pos * rho[2],
            w.w_rot * om[0],  w.w_rot * om[1],  w.w_rot * om[2]};
  T cost = T(0.5) * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3] + r[4] * r[4] + r[5] * r[5]);
  T u1[3], u2[3];
  cross3(om, te, u1);
  cross3(om, u1, u2);
  T J[NZ][6];
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    const int i = k / 2;
    T rel[3] = {pc[0] - Pi[i][0], pc[1] - Pi[i][1], pc[2] - Pi[i][2]};
    T dp[3], Jv[3], Jw[3];
    cross3(Wc[k], rel, dp);
    dp[0] += Pc[k][0];
    dp[1] += Pc[k][1];
    dp[2] += Pc[k][2];
    mtv3(Rc, dp, Jv);
    mtv3(Rc, Wc[k], Jw);
    // y = V^-1 Jw
    T t1[3], t2[3], y[3];
    cross3(om, Jw, t1);
    cross3(om, t1, t2);
    y[0] = Jw[0] - T(0.5) * t1[0] + gam * t2[0];
    y[1] = Jw[1] - T(0.5) * t1[1] + gam * t2[1];
    y[2] = Jw[2] - T(0.5) * t1[2] + gam * t2[2];
    // x = Jv - t x Jw ; Vx = V^-1 x
    T x[3], Vx[3];
    cross3(te, Jw, t1);
    x[0] = Jv[0] - t1[0];
    x[1] = Jv[1] - t1[1];
    x[2] = Jv[2] - t1[2];
    cross3(om, x, t1);
    cross3(om, t1, t2);
    Vx[0] = x[0] - T(0.5) * t1[0] + gam * t2[0];
    Vx[1] = x[1] - T(0.5) * t1[1] + gam * t2[1];
    Vx[2] = x[2] - T(0.5) * t1[2] + gam * t2[2];
    // N y
    T ty[3], u1y[3], wty[3];
    cross3(te, y, ty);
    cross3(u1, y, u1y);
    cross3(om, ty, wty);
    T s2 = T(2) * dgam * dot3(om, y);
    T Ny[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) Ny[m] = T(0.5) * ty[m] + s2 * u2[m] - gam * (u1y[m] + wty[m]);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      J[k][m] = -w.w_pos * (Vx[m] + Ny[m]);
      J[k][3 + m] = -w.w_rot * y[m];
    }
  }
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < 6; ++m) acc += J[k][m] * r[m];
    g[k] = acc;
#pragma unroll
    for (int l = 0; l <= k; ++l) {
      T h = T(0);
#pragma unroll
      for (int m = 0; m < 6; ++m) h += J[k][m] * J[l][m];
      Hp[tri(k, l)] = h;
    }
  }
  bounds_normal_eq<NS, NZ>(rb, w, z, 0, Hp, g, cost);
  return cost;
}

// ---------------------------------------------------------------------------
// Dense Cholesky solve of a packed lower SPD matrix in registers.
// Returns false on a non-positive (or non-finite) pivot.
// ---------------------------------------------------------------------------

template <int N, typename T>
CR_HD bool chol_solve(T* A, T* x) {
  bool ok = true;
  T inv[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T d = A[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= A[tri(j, k)] * A[tri(j, k)];
    ok = ok && (d > T(0));
    const T ljj = tsqrt(d > T(0) ? d : T(1));
    inv[j] = trcp(ljj);
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T v = A[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= A[tri(i, k)] * A[tri(j, k)];
      A[tri(i, j)] = v * inv[j];
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T v = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= A[tri(i, k)] * x[k];
    x[i] = v * inv[i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T v = x[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) v -= A[tri(k, i)] * x[k];
    x[i] = v * inv[i];
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Levenberg-Marquardt with backtracking line search on one IK seed (Sec. IV-C):
//   (H + lambda D) delta = -g, D = diag(max(H_jj, 1e-12));
//   first alpha in 1, 1/2, ... with cost(z + alpha delta) <= cost + 1e-4 alpha g.delta;
//   lambda /= 10 when the full step is taken, *= 10 when every trial fails.
// ---------------------------------------------------------------------------

template <typename T>
struct LMOpts {
  int ls_max;
  T lam_min, lam_max;
};

template <int NS, typename T>
CR_HD void lm_ik(const RobotT<T>& rb, const WeightsT<T>& w, const T* Tt, T* z, T& lam, int iters, const LMOpts<T>& o,
                 bool& failed, int& trials) {
  constexpr int NZ = 2 * NS;
  constexpr int NP = NZ * (NZ + 1) / 2;
  for (int it = 0; it < iters; ++it) {
    T Hp[NP], g[NZ], dl[NZ];
    const T c0 = ik_normal_eq<NS>(rb, w, Tt, z, Hp, g);
    if (!tfinite(c0)) {
      failed = true;
      break;
    }
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      const T hj = Hp[tri(j, j)];
      Hp[tri(j, j)] = hj + lam * (hj > T(1e-12) ? hj : T(1e-12));
      dl[j] = -g[j];
    }
    if (!chol_solve<NZ>(Hp, dl)) {
      if (!(lam < o.lam_max)) break;  // z and lambda would repeat: every later iteration is this one
      lam = lam * T(10) < o.lam_max ? lam * T(10) : o.lam_max;
      continue;
    }
    T gd = T(0);
#pragma unroll
    for (int j = 0; j < NZ; ++j) gd += g[j] * dl[j];
    T alpha = T(1);
    int acc = -1;
    T zt[NZ];
    for (int tr = 0; tr < o.ls_max; ++tr) {
#pragma unroll
      for (int j = 0; j < NZ; ++j) zt[j] = z[j] + alpha * dl[j];
      const T c = ik_cost<NS>(rb, w, Tt, zt, (T*)nullptr);
      ++trials;
      if (c <= c0 + T(1e-4) * alpha * gd) {
        acc = tr;
        break;
      }
      alpha *= T(0.5);
    }
    if (acc >= 0) {
#pragma unroll
      for (int j = 0; j < NZ; ++j) z[j] = zt[j];
      if (acc == 0) lam = lam / T(10) > o.lam_min ? lam / T(10) : o.lam_min;
    } else {
      if (!(lam < o.lam_max)) break;  // rejected at the largest damping: a fixed point of the iteration
      lam = lam * T(10) < o.lam_max ? lam * T(10) : o.lam_max;
    }
  }
}

}  // namespace crk

// ===========================================================================
// Cost and gradient by adjoint sweep (eq. 8-17) for one configuration.
//
// Forward pass: chain the segments, keep for every segment j and coordinate k
// the spatial twist column (W_jk, Pd_jk) -- the rotation axis rate and the
// displacement rate of segment j's end -- and the end position pe_j.  A force f
// applied at a point x distal to segment j's end contributes
//   dC/dz_jk = W_jk . ((x - pe_j) x f) + Pd_jk . f,
// so every distal force/torque can be accumulated into one wrench per segment
// (force, moment about the origin) and swept back from the tip in O(n).
// Backbone points inside segment j add their own-arc term directly.
// ===========================================================================

namespace crk {

// Backbone point at arc fraction sg of a segment with bending coordinates (a, b),
// s = a^2 + b^2, length L, whose base frame is (Rc, pc); rounded to T.
template <typename TC, typename T>
CR_HD void seg_point(const TC* Rc, const TC* pc, TC a, TC b, TC L, TC s, TC sg, T* out) {
  ArcCoef<TC> ck = arc_coef<TC, false>(sg * sg * s);
  const TC sL = sg * L;
  TC dk[3] = {sL * ck.A * (sg * a), sL * ck.A * (sg * b), sL * ck.B}, x[3];
  mv3(Rc, dk, x);
  out[0] = (T)(pc[0] + x[0]);
  out[1] = (T)(pc[1] + x[1]);
  out[2] = (T)(pc[2] + x[2]);
}

template <int NS, typename T, bool EXT = false>
struct Fwd {
  static constexpr int NC = EXT ? 3 : 2, NZ = NC * NS;
  T W[NZ][3], Pd[NZ][3], pe[NS][3];  // twist columns and segment ends
  T R[9], p[3];                      // tip frame
  T F[NS][3], Mo[NS][3];             // force and moment about the origin from points of segment i
  T gz[NZ];                          // direct gradient terms (own arc, bounds)
};

// Convex polytopes in half-space form (convex obstacles): polytope j of a problem
// is the intersection of its F half-spaces n.x <= d, plane f of polytope j with
// component c (nx, ny, nz, d; unit normals) at pl[c * ld + j * F + f].  Signed
// distance sd(x) = max_f (n_f . x - d_f): exact inside the polytope and in the
// region of each face outside it, below the distance near edges and corners
// outside; it is 1-Lipschitz (unit normals).  Unused planes are n = 0, d large.
template <typename TS>
struct PolyArgs {
  const TS* pl;
  int64_t ld;
  int NP, F;
};

// sd of x to polytope j; *arg = the plane of the first largest value
template <typename TC, typename TS>
CR_HD TC poly_sd(const PolyArgs<TS>& po, int j, const TC* x, int* arg) {
  TC s = TC(0);
  int a = 0;
  for (int f = 0; f < po.F; ++f) {
    const int64_t col = (int64_t)j * po.F + f;
    const TC v = (TC)po.pl[col] * x[0] + (TC)po.pl[po.ld + col] * x[1] + (TC)po.pl[2 * po.ld + col] * x[2] -
                 (TC)po.pl[3 * po.ld + col];
    if (f == 0 || v > s) {
      s = v;
      a = f;
    }
  }
  if (arg) *arg = a;
  return s;
}

// Sphere m, component c (cx, cy, cz, radius) is read as sph[m * ms + c * cs].
// zd (NC NS, FP64) or NULL: the coordinates in FP64 when the caller has them (z
// is their rounding to T); a TC chain starts from them.
// TC is the type of the chained transforms, the backbone points and the bound
// hinges.  Every kernel chains in its own type (FP32 kernels in FP32: a clearance
// violation then carries the FP32 error of the point positions, about
// 8 n u32 sum(L), which the FP32 parity tests allow for).  The pair rejection test
// runs in T (with a relative slack when TC is wider); active pairs are measured
// in TC.
// Self contact (eq. 10) of the points of segment j against those of every
// segment m <= j - 2: residual sq_coll max(0, margin + r_j + r_m - |q - p|) per
// pair of points q (segment j) and p (segment m).  Segment m's base frame is
// (Rb[m], pb[m]) and sb[m] = (a, b, L).  With GRAD the pair's force acts on q and,
// opposite, on p: recorded as point forces of both segments (swept back by
// config_reverse) plus their own-arc terms.  Every point lies within L / 2 of its
// segment's arc midpoint, so a segment pair whose midpoints are farther apart than
// (L_j + L_m) / 2 + the reach is skipped whole.
template <int NS, typename T, bool GRAD, typename TC, bool EXT>
CR_HD T self_contact(const RobotT<T>& rb, const WeightsT<T>& w, int j, const TC (*Rb)[9], const TC (*pb)[3],
                     const TC (*sb)[3], Fwd<NS, T, EXT>& f) {
  constexpr int NC = EXT ? 3 : 2;
  T cost = T(0);
  const int K = rb.K;
  const TC rj = sizeof(TC) == 8 ? (TC)rb.rd[j] : (TC)rb.r[j];
  const TC marg = sizeof(TC) == 8 ? (TC)w.margind : (TC)w.margin;
  const TC sqc = (TC)w.sq_coll;
  const TC aj = sb[j][0], bj = sb[j][1], Lj = sb[j][2], sj = aj * aj + bj * bj;
  TC midj[3];
  seg_point(Rb[j], pb[j], aj, bj, Lj, sj, TC(0.5), midj);
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    if (m + 2 > j) continue;
    const TC am = sb[m][0], bm = sb[m][1], Lm = sb[m][2], sm = am * am + bm * bm;
    const TC rm = sizeof(TC) == 8 ? (TC)rb.rd[m] : (TC)rb.r[m];
    const TC reach = rj + rm + marg;
    {
      TC midm[3];
      seg_point(Rb[m], pb[m], am, bm, Lm, sm, TC(0.5), midm);
      const TC e0 = midj[0] - midm[0], e1 = midj[1] - midm[1], e2 = midj[2] - midm[2];
      const TC lim = (TC(0.5) * (Lj + Lm) + reach) * TC(1.0001);
      if (!(e0 * e0 + e1 * e1 + e2 * e2 < lim * lim)) continue;
    }
    for (int l = 1; l <= K; ++l) {
      const TC sq = TC(l) / TC(K);
      ArcCoef<TC> cq = arc_coef<TC, GRAD>(sq * sq * sj);
      const TC qa = sq * aj, qb = sq * bj, qL = sq * Lj;
      TC dq[3] = {qL * cq.A * qa, qL * cq.A * qb, qL * cq.B}, q[3];
      mv3(Rb[j], dq, q);
      q[0] += pb[j][0];
      q[1] += pb[j][1];
      q[2] += pb[j][2];
      for (int k = 1; k <= K; ++k) {
        const TC sp = TC(k) / TC(K);
        ArcCoef<TC> cp = arc_coef<TC, GRAD>(sp * sp * sm);
        const TC pa = sp * am, pbb = sp * bm, pL = sp * Lm;
        TC dp[3] = {pL * cp.A * pa, pL * cp.A * pbb, pL * cp.B}, pt[3];
        mv3(Rb[m], dp, pt);
        pt[0] += pb[m][0];
        pt[1] += pb[m][1];
        pt[2] += pb[m][2];
        const TC d0 = q[0] - pt[0], d1 = q[1] - pt[1], d2 = q[2] - pt[2];
        const TC dist = tsqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const TC viol = reach - dist;
        if (!(viol > TC(0))) continue;
        const TC rr = sqc * viol;
        cost += (T)(TC(0.5) * rr * rr);
        if (GRAD) {
          // d(1/2 r^2)/dq = -sq_coll r n, n = (q - p)/|q - p| (+z when coincident); -that on p
          const TC sc = dist > TC(0) ? -sqc * rr / dist : TC(0);
          const TC fq[3] = {sc * d0, sc * d1, dist > TC(0) ? sc * d2 : -sqc * rr};
          TC mq[3], mp[3], qq[3], qp[3];
          cross3(q, fq, mq);
          cross3(pt, fq, mp);
          mtv3(Rb[j], fq, qq);
          mtv3(Rb[m], fq, qp);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            f.F[j][c] += (T)fq[c];
            f.Mo[j][c] += (T)mq[c];
            f.F[m][c] -= (T)fq[c];
            f.Mo[m][c] -= (T)mp[c];
          }
          const TC daq[3] = {qL * (cq.A + TC(2) * qa * qa * cq.Ap), qL * TC(2) * qa * qb * cq.Ap, qL * TC(2) * qa * cq.Bp};
          const TC dbq[3] = {qL * TC(2) * qa * qb * cq.Ap, qL * (cq.A + TC(2) * qb * qb * cq.Ap), qL * TC(2) * qb * cq.Bp};
          const TC dap[3] = {pL * (cp.A + TC(2) * pa * pa * cp.Ap), pL * TC(2) * pa * pbb * cp.Ap, pL * TC(2) * pa * cp.Bp};
          const TC dbp[3] = {pL * TC(2) * pa * pbb * cp.Ap, pL * (cp.A + TC(2) * pbb * pbb * cp.Ap), pL * TC(2) * pbb * cp.Bp};
          f.gz[NC * j] += (T)(sq * dot3(qq, daq));
          f.gz[NC * j + 1] += (T)(sq * dot3(qq, dbq));
          f.gz[NC * m] -= (T)(sp * dot3(qp, dap));
          f.gz[NC * m + 1] -= (T)(sp * dot3(qp, dbp));
          if constexpr (EXT) {
            const TC deq[3] = {sq * cq.A * qa, sq * cq.A * qb, sq * cq.B};
            const TC dep[3] = {sp * cp.A * pa, sp * cp.A * pbb, sp * cp.B};
            f.gz[NC * j + 2] += (T)dot3(qq, deq);
            f.gz[NC * m + 2] -= (T)dot3(qp, dep);
          }
        }
      }
    }
  }
  return cost;
}

// POLY: clearance rows against the convex polytopes of po as well.
template <int NS, typename T, bool GRAD, typename TC = T, typename TS = T, bool EXT = false, bool SELF = false,
          bool POLY = false>
CR_HD T config_forward(const RobotT<T>& rb, const WeightsT<T>& w, const T* z, const TS* sph, int M, int64_t ms,
                       int64_t cs, Fwd<NS, T, EXT>& f, const double* zd = nullptr,
                       const PolyArgs<TS>& po = PolyArgs<TS>{nullptr, 0, 0, 0}) {
  constexpr int NC = EXT ? 3 : 2;
  T cost = T(0);
  TC Rc[9], pc[3];
  // self contact: base frame, bending and length of every segment, for the points
  // of segments two or more behind the current one
  TC Rb[SELF ? NS : 1][9], pb[SELF ? NS : 1][3], sb[SELF ? NS : 1][3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = (k % 4 == 0) ? TC(1) : TC(0);
  pc[0] = pc[1] = pc[2] = TC(0);
  if (GRAD) {
#pragma unroll
    for (int k = 0; k < NC * NS; ++k) f.gz[k] = T(0);
  }
  const int K = rb.K;
  const T slack = sizeof(T) < sizeof(TC) ? T(1.0001) : T(1);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const T a = z[NC * i], b = z[NC * i + 1];
    const TC ac = zd ? (TC)zd[NC * i] : (TC)a, bc = zd ? (TC)zd[NC * i + 1] : (TC)b;
    TC Lc = sizeof(TC) == 8 ? (TC)rb.Ld[i] : (TC)rb.L[i];
    if constexpr (EXT) Lc += zd ? (TC)zd[NC * i + 2] : (TC)z[NC * i + 2];
    const TC s = ac * ac + bc * bc;
    if (GRAD) {
#pragma unroll
      for (int c = 0; c < 3; ++c) f.F[i][c] = f.Mo[i][c] = T(0);
    }
    if constexpr (SELF) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Rb[i][k] = Rc[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) pb[i][k] = pc[k];
      sb[i][0] = ac;
      sb[i][1] = bc;
      sb[i][2] = Lc;
      cost += self_contact<NS, T, GRAD, TC, EXT>(rb, w, i, Rb, pb, sb, f);
    }
    // backbone points of this segment against every sphere (eq. 10).  Every point
    // lies within L_i / 2 of the arc midpoint (arc length bounds the chord), so a
    // sphere farther than L_i / 2 + R + r_i + margin from it is skipped for the
    // whole segment without changing the cost.
    if (M > 0) {
      const TC ri = sizeof(TC) == 8 ? (TC)rb.rd[i] : (TC)rb.r[i];
      const TC marg = sizeof(TC) == 8 ? (TC)w.margind : (TC)w.margin;
      const TC sqc = (TC)w.sq_coll;
      const T rf = (T)(ri + marg);
      T xmf[3];
      seg_point(Rc, pc, ac, bc, Lc, s, TC(0.5), xmf);
      const T Lf = (T)Lc;
      const T half = T(0.5) * Lf;
      for (int m = 0; m < M; ++m) {
        const TS* sp = sph + m * ms;
        const T sm[4] = {(T)sp[0], (T)sp[cs], (T)sp[2 * cs], (T)sp[3 * cs]};
        {
          const T e0 = xmf[0] - sm[0], e1 = xmf[1] - sm[1], e2 = xmf[2] - sm[2];
          const T rq = (sm[3] + rf + half) * T(1.0001);
          if (!(e0 * e0 + e1 * e1 + e2 * e2 < rq * rq)) continue;
        }
        const TC cx = (TC)sp[0], cy = (TC)sp[cs], cz = (TC)sp[2 * cs];
        const TC reach = (TC)sp[3 * cs] + ri + marg;
        const T rq = (sm[3] + rf) * slack;
        // runs of at most 8 points, each skipped when the ball around its middle
        // arc point (radius: half the run's arc length) misses the sphere
        for (int k0 = 1; k0 <= K; k0 += 8) {
          const int k1 = k0 + 7 < K ? k0 + 7 : K;
          {
            T xr[3];
            seg_point(Rc, pc, ac, bc, Lc, s, TC(k0 + k1) * TC(0.5) / TC(K), xr);
            const T e0 = xr[0] - sm[0], e1 = xr[1] - sm[1], e2 = xr[2] - sm[2];
            const T rr = (sm[3] + rf + T(k1 - k0) * T(0.5) / T(K) * Lf) * T(1.0001);
            if (!(e0 * e0 + e1 * e1 + e2 * e2 < rr * rr)) continue;
          }
          for (int k = k0; k <= k1; ++k) {
            const TC sg = TC(k) / TC(K);
            ArcCoef<TC> ck = arc_coef<TC, GRAD>(sg * sg * s);
            const TC sa = sg * ac, sb = sg * bc, sL = sg * Lc;
            TC dk[3] = {sL * ck.A * sa, sL * ck.A * sb, sL * ck.B};
            TC x[3];
            mv3(Rc, dk, x);
            x[0] += pc[0];
            x[1] += pc[1];
            x[2] += pc[2];
            const TC d0 = x[0] - cx, d1 = x[1] - cy, d2 = x[2] - cz;
            {
              const T e0 = (T)d0, e1 = (T)d1, e2 = (T)d2;
              if (!(e0 * e0 + e1 * e1 + e2 * e2 < rq * rq)) continue;
            }
            const TC dist = tsqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const TC viol = reach - dist;  // margin - (dist - R - r)
            if (!(viol > TC(0))) continue;
            const TC rr = sqc * viol;
            cost += (T)(TC(0.5) * rr * rr);
            if (GRAD) {
              // d(1/2 r^2)/dx = -sq_coll r n,  n = (x - c)/|x - c|  (+z when coincident)
              const TC sc = dist > TC(0) ? -sqc * rr / dist : TC(0);
              const TC fx[3] = {sc * d0, sc * d1, dist > TC(0) ? sc * d2 : -sqc * rr};
  #pragma unroll
              for (int q = 0; q < 3; ++q) f.F[i][q] += (T)fx[q];
              TC mx[3];
              cross3(x, fx, mx);
  #pragma unroll
              for (int q = 0; q < 3; ++q) f.Mo[i][q] += (T)mx[q];
              // own arc: x = pc + Rc d(sg a, sg b, sg L)
              TC q[3];
              mtv3(Rc, fx, q);
              const TC dda[3] = {sL * (ck.A + TC(2) * sa * sa * ck.Ap), sL * TC(2) * sa * sb * ck.Ap, sL * TC(2) * sa * ck.Bp};
              const TC ddb[3] = {sL * TC(2) * sa * sb * ck.Ap, sL * (ck.A + TC(2) * sb * sb * ck.Ap), sL * TC(2) * sb * ck.Bp};
              f.gz[NC * i] += (T)(sg * dot3(q, dda));
              f.gz[NC * i + 1] += (T)(sg * dot3(q, ddb));
              if constexpr (EXT) {
                // the point moves with the length: dx/de = Rc sg (A sa, A sb, B)
                const TC dde[3] = {sg * ck.A * sa, sg * ck.A * sb, sg * ck.B};
                f.gz[NC * i + 2] += (T)dot3(q, dde);
              }
            }
          }
        }
      }
    }
    if constexpr (POLY) {
      // backbone points of this segment against every convex polytope: sd is
      // 1-Lipschitz and every point lies within L_i / 2 of the arc midpoint, so a
      // polytope farther than L_i / 2 + r_i + margin from it is skipped
      const TC ri = sizeof(TC) == 8 ? (TC)rb.rd[i] : (TC)rb.r[i];
      const TC marg = sizeof(TC) == 8 ? (TC)w.margind : (TC)w.margin;
      const TC sqc = (TC)w.sq_coll;
      TC xm[3];
      seg_point(Rc, pc, ac, bc, Lc, s, TC(0.5), xm);
      for (int jp = 0; jp < po.NP; ++jp) {
        if (poly_sd<TC>(po, jp, xm, (int*)nullptr) - TC(0.5) * Lc - ri - marg > TC(1e-6)) continue;
        for (int k = 1; k <= K; ++k) {
          const TC sg = TC(k) / TC(K);
          ArcCoef<TC> ck = arc_coef<TC, GRAD>(sg * sg * s);
          const TC sa = sg * ac, sb = sg * bc, sL = sg * Lc;
          TC dk[3] = {sL * ck.A * sa, sL * ck.A * sb, sL * ck.B};
          TC x[3];
          mv3(Rc, dk, x);
          x[0] += pc[0];
          x[1] += pc[1];
          x[2] += pc[2];
          int fa;
          const TC viol = marg + ri - poly_sd<TC>(po, jp, x, &fa);
          if (!(viol > TC(0))) continue;
          const TC rr = sqc * viol;
          cost += (T)(TC(0.5) * rr * rr);
          if (GRAD) {
            // d(1/2 r^2)/dx = -sq_coll r n_f of the plane that attains sd
            const int64_t col = (int64_t)jp * po.F + fa;
            const TC sc = -sqc * rr;
            const TC fx[3] = {sc * (TC)po.pl[col], sc * (TC)po.pl[po.ld + col], sc * (TC)po.pl[2 * po.ld + col]};
#pragma unroll
            for (int q = 0; q < 3; ++q) f.F[i][q] += (T)fx[q];
            TC mx[3];
            cross3(x, fx, mx);
#pragma unroll
            for (int q = 0; q < 3; ++q) f.Mo[i][q] += (T)mx[q];
            TC q[3];
            mtv3(Rc, fx, q);
            const TC dda[3] = {sL * (ck.A + TC(2) * sa * sa * ck.Ap), sL * TC(2) * sa * sb * ck.Ap, sL * TC(2) * sa * ck.Bp};
            const TC ddb[3] = {sL * TC(2) * sa * sb * ck.Ap, sL * (ck.A + TC(2) * sb * sb * ck.Ap), sL * TC(2) * sb * ck.Bp};
            f.gz[NC * i] += (T)(sg * dot3(q, dda));
            f.gz[NC * i + 1] += (T)(sg * dot3(q, ddb));
            if constexpr (EXT) {
              const TC dde[3] = {sg * ck.A * sa, sg * ck.A * sb, sg * ck.B};
              f.gz[NC * i + 2] += (T)dot3(q, dde);
            }
          }
        }
      }
    }
    ArcCoef<TC> c = arc_coef<TC, GRAD>(s);
    TC Ri[9], di[3];
    seg_R_d(ac, bc, Lc, c, Ri, di);
    if (GRAD) {
      TC wa[3] = {-c.C * ac * bc, TC(1) - c.C * bc * bc, -c.A * bc};
      TC wb[3] = {c.C * ac * ac - TC(1), c.C * ac * bc, c.A * ac};
      TC dda[3] = {Lc * (c.A + TC(2) * ac * ac * c.Ap), Lc * TC(2) * ac * bc * c.Ap, Lc * TC(2) * ac * c.Bp};
      TC ddb[3] = {Lc * TC(2) * ac * bc * c.Ap, Lc * (c.A + TC(2) * bc * bc * c.Ap), Lc * TC(2) * bc * c.Bp};
      TC t0[3];
      mv3(Rc, wa, t0);
#pragma unroll
      for (int q = 0; q < 3; ++q) f.W[NC * i][q] = (T)t0[q];
      mv3(Rc, wb, t0);
#pragma unroll
      for (int q = 0; q < 3; ++q) f.W[NC * i + 1][q] = (T)t0[q];
      mv3(Rc, dda, t0);
#pragma unroll
      for (int q = 0; q < 3; ++q) f.Pd[NC * i][q] = (T)t0[q];
      mv3(Rc, ddb, t0);
#pragma unroll
      for (int q = 0; q < 3; ++q) f.Pd[NC * i + 1][q] = (T)t0[q];
      if constexpr (EXT) {
        // the extension moves the segment's end along d_i / L_i and does not rotate it
        const TC dde[3] = {c.A * ac, c.A * bc, c.B};
        mv3(Rc, dde, t0);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          f.W[NC * i + 2][q] = T(0);
          f.Pd[NC * i + 2][q] = (T)t0[q];
        }
      }
    }
    TC q[3], Rn[9];
    mv3(Rc, di, q);
    pc[0] += q[0];
    pc[1] += q[1];
    pc[2] += q[2];
    mm3(Rc, Ri, Rn);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = Rn[k];
    if (GRAD) {
      f.pe[i][0] = (T)pc[0];
      f.pe[i][1] = (T)pc[1];
      f.pe[i][2] = (T)pc[2];
    }
    // bounds (eq. 9): tendon hinges and bending hinge, in the chain's type
    {
      TC ru[3], sg[3], rth;
      bound_residuals<TC>(rb, w, i, ac, bc, ru, sg, &rth);
      const TC cb = TC(0.5) * (ru[0] * ru[0] + ru[1] * ru[1] + ru[2] * ru[2] + rth * rth);
      cost += (T)cb;
      if (GRAD) {
        TC ga = TC(0), gb = TC(0);
        const TC ri = sizeof(TC) == 8 ? (TC)rb.rd[i] : (TC)rb.r[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (ru[j] > TC(0)) {
            TC ja, jb;
            lift_row(j, ri, &ja, &jb);
            ga += sg[j] * (TC)w.sq_lim * ja * ru[j];
            gb += sg[j] * (TC)w.sq_lim * jb * ru[j];
          }
        }
        if (rth > TC(0)) {
          const TC ith = trcp(tsqrt(s));
          ga += (TC)w.sq_curv * ac * ith * rth;
          gb += (TC)w.sq_curv * bc * ith * rth;
        }
        f.gz[NC * i] += (T)ga;
        f.gz[NC * i + 1] += (T)gb;
      }
      if constexpr (EXT) {
        TC se;
        const TC ed = zd ? (TC)zd[NC * i + 2] : (TC)z[NC * i + 2];
        const TC rl = length_residual<TC>(rb, w, i, ed, &se);
        cost += (T)(TC(0.5) * rl * rl);
        if (GRAD && rl > TC(0)) f.gz[NC * i + 2] += (T)(se * (TC)w.sq_lim * rl);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) f.R[k] = (T)Rc[k];
  f.p[0] = (T)pc[0];
  f.p[1] = (T)pc[1];
  f.p[2] = (T)pc[2];
  return cost;
}

// Pose objective log(T_ee^-1 T_t) with weights (eq. 8/16): returns 1/2 |r|^2 and, if
// GRAD, the tip wrench (world force f, world torque tau) equivalent to the
// gradient: dC/dxi_body = (lambda_v, lambda_w) = M^T r, f = R lambda_v, tau = R lambda_w.
template <typename T, bool GRAD>
CR_HD T pose_term(const WeightsT<T>& w, const T* R, const T* p, const T* Tt, T* f, T* tau) {
  T Re[9], te[3], om[3], rho[3], gam, dgam = T(0);
  relative_pose(R, p, Tt, Re, te);
  log_se3<T, GRAD>(Re, te, om, rho, &gam, &dgam);
  const T rr[3] = {w.w_pos * rho[0], w.w_pos * rho[1], w.w_pos * rho[2]};
  const T ro[3] = {w.w_rot * om[0], w.w_rot * om[1], w.w_rot * om[2]};
  const T cost = T(0.5) * (dot3(rr, rr) + dot3(ro, ro));
  if (GRAD) {
    // V^-T x = x + w x x / 2 + gamma w x (w x x)
    auto vit = [&](const T* x, T* y) {
      T t1[3], t2[3];
      cross3(om, x, t1);
      cross3(om, t1, t2);
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c] = x[c] + T(0.5) * t1[c] + gam * t2[c];
    };
    T u1[3], u2[3];
    cross3(om, te, u1);
    cross3(om, u1, u2);
    // N^T x = -t x x / 2 + 2 gamma' (u2 . x) w + gamma u1 x x - gamma t x (w x x)
    T tx[3], u1x[3], wx[3], twx[3], Nt[3];
    cross3(te, rr, tx);
    cross3(u1, rr, u1x);
    cross3(om, rr, wx);
    cross3(te, wx, twx);
    const T s2 = T(2) * dgam * dot3(u2, rr);
#pragma unroll
    for (int c = 0; c < 3; ++c) Nt[c] = T(-0.5) * tx[c] + s2 * om[c] + gam * (u1x[c] - twx[c]);
    T a1[3], a2[3], a3[3], ta2[3], lv[3], lw[3];
    vit(Nt, a1);
    vit(rr, a2);
    vit(ro, a3);
    cross3(te, a2, ta2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lv[c] = -w.w_pos * a2[c];
      lw[c] = -w.w_pos * (a1[c] + ta2[c]) - w.w_rot * a3[c];
    }
    mv3(R, lv, f);
    mv3(R, lw, tau);
  }
  return cost;
}

// Reverse sweep: gz += contributions of the tip wrench (f_tip, tau_tip) and of
// the per-segment point forces recorded in the forward pass.
template <int NS, typename T, bool EXT = false>
CR_HD void config_reverse(const Fwd<NS, T, EXT>& f, const T* f_tip, const T* tau_tip, T* gz) {
  constexpr int NC = EXT ? 3 : 2;
  T Fd[3] = {f_tip[0], f_tip[1], f_tip[2]};
  T Md[3];
  cross3(f.p, f_tip, Md);
  Md[0] += tau_tip[0];
  Md[1] += tau_tip[1];
  Md[2] += tau_tip[2];
#pragma unroll
  for (int j = NS - 1; j >= 0; --j) {
    T pf[3], mom[3];
    cross3(f.pe[j], Fd, pf);
    mom[0] = Md[0] - pf[0];
    mom[1] = Md[1] - pf[1];
    mom[2] = Md[2] - pf[2];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      gz[NC * j + c] = f.gz[NC * j + c] + dot3(f.W[NC * j + c], mom) + dot3(f.Pd[NC * j + c], Fd);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Fd[c] += f.F[j][c];
      Md[c] += f.Mo[j][c];
    }
  }
}

// dC/du from dC/dz for one segment: a = (u1 + u2 - 2 u0)/(3r), b = (u2 - u1)/(sqrt(3) r).
template <typename T>
CR_HD void gz_to_gu(T ga, T gb, T r, T* gu) {
  const T i3r = T(1) / (T(3) * r), is3r = T(1) / (T(1.7320508075688772935) * r);
  gu[0] = T(-2) * ga * i3r;
  gu[1] = ga * i3r - gb * is3r;
  gu[2] = ga * i3r + gb * is3r;
}

}  // namespace crk

// ===========================================================================
// Gauss-Newton blocks of one configuration for the trajectory solvers: pose
// rows (if a target is given), bound rows, clearance rows of every active
// point/sphere pair, and the tip position with its Jacobian (for the
// path-length term, which couples neighbouring waypoints).
// ===========================================================================

namespace crk {

// Adds the 6 pose rows of log(T_ee^-1 T_t) to Hp, g and returns their cost.
// Columns: for coordinate k the spatial twist (W[k], dp[k]) of the tip, with
// dp already including the lever arm to the tip.
template <int NZ, typename T>
CR_HD T pose_rows(const WeightsT<T>& w, const T* Rc, const T* pc, T (*W)[3], T (*dp)[3], const T* Tt, T* Hp,
                  T* g) {
  T Re[9], te[3], om[3], rho[3], gam, dgam;
  relative_pose(Rc, pc, Tt, Re, te);
  log_se3<T, true>(Re, te, om, rho, &gam, &dgam);
  const T r[6] = {w.w_pos * rho[0], w.w_pos * rho[1], w.w_pos * rho[2],
                  w.w_rot * om[0],  w.w_rot * om[1],  w.w_rot * om[2]};
  T u1[3], u2[3];
  cross3(om, te, u1);
  cross3(om, u1, u2);
  T J[NZ][6];
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    T Jv[3], Jw[3], t1[3], t2[3], y[3], x[3], Vx[3];
    mtv3(Rc, dp[k], Jv);
    mtv3(Rc, W[k], Jw);
    cross3(om, Jw, t1);
    cross3(om, t1, t2);
#pragma unroll
    for (int m = 0; m < 3; ++m) y[m] = Jw[m] - T(0.5) * t1[m] + gam * t2[m];
    cross3(te, Jw, t1);
#pragma unroll
    for (int m = 0; m < 3; ++m) x[m] = Jv[m] - t1[m];
    cross3(om, x, t1);
    cross3(om, t1, t2);
#pragma unroll
    for (int m = 0; m < 3; ++m) Vx[m] = x[m] - T(0.5) * t1[m] + gam * t2[m];
    T ty[3], u1y[3], wty[3];
    cross3(te, y, ty);
    cross3(u1, y, u1y);
    cross3(om, ty, wty);
    const T s2 = T(2) * dgam * dot3(om, y);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      J[k][m] = -w.w_pos * (Vx[m] + T(0.5) * ty[m] + s2 * u2[m] - gam * (u1y[m] + wty[m]));
      J[k][3 + m] = -w.w_rot * y[m];
    }
  }
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < 6; ++m) acc += J[k][m] * r[m];
    g[k] += acc;
#pragma unroll
    for (int l = 0; l <= k; ++l) {
      T h = T(0);
#pragma unroll
      for (int m = 0; m < 6; ++m) h += J[k][m] * J[l][m];
      Hp[tri(k, l)] += h;
    }
  }
  return T(0.5) * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3] + r[4] * r[4] + r[5] * r[5]);
}

// Hp (packed lower, 2NS), g are overwritten.  ptip[3] and Jp[3][2NS] receive the
// tip position and its Jacobian.  Pose rows against Tt only if pose.  TC is the
// chain type (as in config_forward).
template <int NS, typename T, typename TC, typename TS = T, bool EXT = false, bool SELF = false, bool POLY = false>
CR_HD T local_normal_eq(const RobotT<T>& rb, const WeightsT<T>& w, const T* z, const TS* sph, int M, int64_t ms,
                        int64_t cs, const T* Tt, T* Hp, T* g, T* ptip, T (*Jp)[(EXT ? 3 : 2) * NS], bool pose = true,
                        const PolyArgs<TS>& po = PolyArgs<TS>{nullptr, 0, 0, 0}) {
  constexpr int NC = EXT ? 3 : 2, NZ = NC * NS, NP = NZ * (NZ + 1) / 2;
#pragma unroll
  for (int k = 0; k < NP; ++k) Hp[k] = T(0);
#pragma unroll
  for (int k = 0; k < NZ; ++k) g[k] = T(0);
  T cost = T(0);
  TC Rc[9], pc[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = (k % 4 == 0) ? TC(1) : TC(0);
  pc[0] = pc[1] = pc[2] = TC(0);
  T W[NZ][3], Pd[NZ][3], pe[NS][3];
  TC Rb[SELF ? NS : 1][9], pbs[SELF ? NS : 1][3];  // base frames (self contact)
  const int K = rb.K;
  const T slack = sizeof(T) < sizeof(TC) ? T(1.0001) : T(1);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const TC ac = (TC)z[NC * i], bc = (TC)z[NC * i + 1];
    TC Lc = sizeof(TC) == 8 ? (TC)rb.Ld[i] : (TC)rb.L[i];
    if constexpr (EXT) Lc += (TC)z[NC * i + 2];
    const TC s = ac * ac + bc * bc;
    if constexpr (SELF) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Rb[i][k] = Rc[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) pbs[i][k] = pc[k];
      // self-contact rows (eq. 10): points q of this segment against points p of every
      // segment m <= i - 2; both move rigidly with the segments before m, so only the
      // columns of segments m..i enter the row
#pragma unroll
      for (int m = 0; m < NS; ++m) {
        if (m + 2 > i) continue;
        const TC am = (TC)z[NC * m], bm = (TC)z[NC * m + 1], sm = am * am + bm * bm;
        TC Lm = sizeof(TC) == 8 ? (TC)rb.Ld[m] : (TC)rb.L[m];
        if constexpr (EXT) Lm += (TC)z[NC * m + 2];
        const TC ri = sizeof(TC) == 8 ? (TC)rb.rd[i] : (TC)rb.r[i];
        const TC rm = sizeof(TC) == 8 ? (TC)rb.rd[m] : (TC)rb.r[m];
        const TC reach = ri + rm + (sizeof(TC) == 8 ? (TC)w.margind : (TC)w.margin);
        {
          TC mi[3], mm[3];
          seg_point(Rc, pc, ac, bc, Lc, s, TC(0.5), mi);
          seg_point(Rb[m], pbs[m], am, bm, Lm, sm, TC(0.5), mm);
          const TC e0 = mi[0] - mm[0], e1 = mi[1] - mm[1], e2 = mi[2] - mm[2];
          const TC lim = (TC(0.5) * (Lc + Lm) + reach) * TC(1.0001);
          if (!(e0 * e0 + e1 * e1 + e2 * e2 < lim * lim)) continue;
        }
        for (int l = 1; l <= K; ++l) {
          const TC sq = TC(l) / TC(K);
          ArcCoef<TC> cq = arc_coef<TC, true>(sq * sq * s);
          const TC qa = sq * ac, qb = sq * bc, qL = sq * Lc;
          TC dq[3] = {qL * cq.A * qa, qL * cq.A * qb, qL * cq.B}, q[3];
          mv3(Rc, dq, q);
          q[0] += pc[0];
          q[1] += pc[1];
          q[2] += pc[2];
          for (int k = 1; k <= K; ++k) {
            const TC sp = TC(k) / TC(K);
            ArcCoef<TC> cp = arc_coef<TC, true>(sp * sp * sm);
            const TC pa = sp * am, pbb = sp * bm, pL = sp * Lm;
            TC dp[3] = {pL * cp.A * pa, pL * cp.A * pbb, pL * cp.B}, pt[3];
            mv3(Rb[m], dp, pt);
            pt[0] += pbs[m][0];
            pt[1] += pbs[m][1];
            pt[2] += pbs[m][2];
            const TC d0 = q[0] - pt[0], d1 = q[1] - pt[1], d2 = q[2] - pt[2];
            const TC dist = tsqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const TC viol = reach - dist;
            if (!(viol > TC(0))) continue;
            const T rr = (T)((TC)w.sq_coll * viol);
            TC nv[3];
            if (dist > TC(0)) {
              const TC id = TC(1) / dist;
              nv[0] = d0 * id;
              nv[1] = d1 * id;
              nv[2] = d2 * id;
            } else {
              nv[0] = nv[1] = TC(0);
              nv[2] = TC(1);
            }
            const T nf[3] = {(T)nv[0], (T)nv[1], (T)nv[2]}, qf[3] = {(T)q[0], (T)q[1], (T)q[2]};
            T row[NZ];
#pragma unroll
            for (int c = 0; c < NZ; ++c) row[c] = T(0);
            // segments m .. i-1: q moves rigidly with them (q distal to their ends)
#pragma unroll
            for (int c = 0; c < NS; ++c) {
              if (c >= m && c < i) {
                T xm[3] = {qf[0] - pe[c][0], qf[1] - pe[c][1], qf[2] - pe[c][2]}, c3[3];
                cross3(xm, nf, c3);
#pragma unroll
                for (int e = 0; e < NC; ++e)
                  row[NC * c + e] = -w.sq_coll * (dot3(W[NC * c + e], c3) + dot3(Pd[NC * c + e], nf));
              }
            }
            // own arcs: q within segment i (+), p within segment m (-)
            {
              TC qq[3], qp[3];
              mtv3(Rc, nv, qq);
              mtv3(Rb[m], nv, qp);
              const TC daq[3] = {qL * (cq.A + TC(2) * qa * qa * cq.Ap), qL * TC(2) * qa * qb * cq.Ap, qL * TC(2) * qa * cq.Bp};
              const TC dbq[3] = {qL * TC(2) * qa * qb * cq.Ap, qL * (cq.A + TC(2) * qb * qb * cq.Ap), qL * TC(2) * qb * cq.Bp};
              const TC dap[3] = {pL * (cp.A + TC(2) * pa * pa * cp.Ap), pL * TC(2) * pa * pbb * cp.Ap, pL * TC(2) * pa * cp.Bp};
              const TC dbp[3] = {pL * TC(2) * pa * pbb * cp.Ap, pL * (cp.A + TC(2) * pbb * pbb * cp.Ap), pL * TC(2) * pbb * cp.Bp};
              const TC sqc = (TC)w.sq_coll;
              row[NC * i] = (T)(-sqc * sq * dot3(qq, daq));
              row[NC * i + 1] = (T)(-sqc * sq * dot3(qq, dbq));
              row[NC * m] += (T)(sqc * sp * dot3(qp, dap));
              row[NC * m + 1] += (T)(sqc * sp * dot3(qp, dbp));
              if constexpr (EXT) {
                const TC deq[3] = {sq * cq.A * qa, sq * cq.A * qb, sq * cq.B};
                const TC dep[3] = {sp * cp.A * pa, sp * cp.A * pbb, sp * cp.B};
                row[NC * i + 2] = (T)(-sqc * dot3(qq, deq));
                row[NC * m + 2] += (T)(sqc * dot3(qp, dep));
              }
            }
            cost += T(0.5) * rr * rr;
#pragma unroll
            for (int k1 = 0; k1 < NZ; ++k1) {
              if (k1 >= NC * m && k1 <= NC * i + NC - 1) {
                g[k1] += row[k1] * rr;
#pragma unroll
                for (int k2 = 0; k2 <= k1; ++k2)
                  if (k2 >= NC * m) Hp[tri(k1, k2)] += row[k1] * row[k2];
              }
            }
          }
        }
      }
    }
    if (M > 0) {
      // clearance rows, with the segment-level sphere culling of config_forward
      const TC ri = sizeof(TC) == 8 ? (TC)rb.rd[i] : (TC)rb.r[i];
      const TC marg = sizeof(TC) == 8 ? (TC)w.margind : (TC)w.margin;
      const T rf = (T)(ri + marg);
      T xmf[3];
      seg_point(Rc, pc, ac, bc, Lc, s, TC(0.5), xmf);
      const T Lf = (T)Lc;
      const T half = T(0.5) * Lf;
      for (int m = 0; m < M; ++m) {
        const TS* sp = sph + m * ms;
        const T sm[4] = {(T)sp[0], (T)sp[cs], (T)sp[2 * cs], (T)sp[3 * cs]};
        {
          const T e0 = xmf[0] - sm[0], e1 = xmf[1] - sm[1], e2 = xmf[2] - sm[2];
          const T rq = (sm[3] + rf + half) * T(1.0001);
          if (!(e0 * e0 + e1 * e1 + e2 * e2 < rq * rq)) continue;
        }
        const TC cx = (TC)sp[0], cy = (TC)sp[cs], cz = (TC)sp[2 * cs];
        const TC reach = (TC)sp[3 * cs] + ri + marg;
        const T rq = (sm[3] + rf) * slack;
        // runs of at most 8 points, each skipped when the ball around its middle
        // arc point (radius: half the run's arc length) misses the sphere
        for (int k0 = 1; k0 <= K; k0 += 8) {
          const int k1 = k0 + 7 < K ? k0 + 7 : K;
          {
            T xr[3];
            seg_point(Rc, pc, ac, bc, Lc, s, TC(k0 + k1) * TC(0.5) / TC(K), xr);
            const T e0 = xr[0] - sm[0], e1 = xr[1] - sm[1], e2 = xr[2] - sm[2];
            const T rr = (sm[3] + rf + T(k1 - k0) * T(0.5) / T(K) * Lf) * T(1.0001);
            if (!(e0 * e0 + e1 * e1 + e2 * e2 < rr * rr)) continue;
          }
          for (int k = k0; k <= k1; ++k) {
            const TC sg = TC(k) / TC(K);
            ArcCoef<TC> ck = arc_coef<TC, true>(sg * sg * s);
            const TC sa = sg * ac, sb = sg * bc, sL = sg * Lc;
            TC dk[3] = {sL * ck.A * sa, sL * ck.A * sb, sL * ck.B};
            TC x[3];
            mv3(Rc, dk, x);
            x[0] += pc[0];
            x[1] += pc[1];
            x[2] += pc[2];
            const TC d0 = x[0] - cx, d1 = x[1] - cy, d2 = x[2] - cz;
            {
              const T e0 = (T)d0, e1 = (T)d1, e2 = (T)d2;
              if (!(e0 * e0 + e1 * e1 + e2 * e2 < rq * rq)) continue;
            }
            const TC dist = tsqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const TC viol = reach - dist;
            if (!(viol > TC(0))) continue;
            const T rr = (T)((TC)w.sq_coll * viol);
            const T xf[3] = {(T)x[0], (T)x[1], (T)x[2]};
            // residual sq_coll (reach - |x - c|): row = -sq_coll n^T dx/dz
            T nvec[3];
            if (dist > TC(0)) {
              const TC id = TC(1) / dist;
              nvec[0] = (T)(d0 * id);
              nvec[1] = (T)(d1 * id);
              nvec[2] = (T)(d2 * id);
            } else {
              nvec[0] = nvec[1] = T(0);
              nvec[2] = T(1);
            }
            T row[NZ];
  #pragma unroll
            for (int q = 0; q < NZ; ++q) row[q] = T(0);
  #pragma unroll
            for (int j = 0; j < NS; ++j) {
              if (j < i) {
                T xm[3] = {xf[0] - pe[j][0], xf[1] - pe[j][1], xf[2] - pe[j][2]}, c3[3];
                cross3(xm, nvec, c3);
  #pragma unroll
                for (int c = 0; c < NC; ++c)
                  row[NC * j + c] = -w.sq_coll * (dot3(W[NC * j + c], c3) + dot3(Pd[NC * j + c], nvec));
              }
            }
            {
              TC nq[3] = {(TC)nvec[0], (TC)nvec[1], (TC)nvec[2]}, q[3];
              mtv3(Rc, nq, q);
              const TC dda[3] = {sL * (ck.A + TC(2) * sa * sa * ck.Ap), sL * TC(2) * sa * sb * ck.Ap, sL * TC(2) * sa * ck.Bp};
              const TC ddb[3] = {sL * TC(2) * sa * sb * ck.Ap, sL * (ck.A + TC(2) * sb * sb * ck.Ap), sL * TC(2) * sb * ck.Bp};
              row[NC * i] = (T)(-(TC)w.sq_coll * sg * dot3(q, dda));
              row[NC * i + 1] = (T)(-(TC)w.sq_coll * sg * dot3(q, ddb));
              if constexpr (EXT) {
                const TC dde[3] = {sg * ck.A * sa, sg * ck.A * sb, sg * ck.B};
                row[NC * i + 2] = (T)(-(TC)w.sq_coll * dot3(q, dde));
              }
            }
            cost += T(0.5) * rr * rr;
  #pragma unroll
            for (int k1 = 0; k1 < NZ; ++k1) {
              if (k1 <= NC * i + NC - 1) {
                g[k1] += row[k1] * rr;
  #pragma unroll
                for (int k2 = 0; k2 <= k1; ++k2) Hp[tri(k1, k2)] += row[k1] * row[k2];
              }
            }
          }
        }
      }
    }
    if constexpr (POLY) {
      // convex-polytope rows (culling as in config_forward): residual
      // sq_coll (margin + r_i - sd(x)), row = -sq_coll n_f^T dx/dz
      const TC ri = sizeof(TC) == 8 ? (TC)rb.rd[i] : (TC)rb.r[i];
      const TC marg = sizeof(TC) == 8 ? (TC)w.margind : (TC)w.margin;
      TC xm[3];
      seg_point(Rc, pc, ac, bc, Lc, s, TC(0.5), xm);
      for (int jp = 0; jp < po.NP; ++jp) {
        if (poly_sd<TC>(po, jp, xm, (int*)nullptr) - TC(0.5) * Lc - ri - marg > TC(1e-6)) continue;
        for (int k = 1; k <= K; ++k) {
          const TC sg = TC(k) / TC(K);
          ArcCoef<TC> ck = arc_coef<TC, true>(sg * sg * s);
          const TC sa = sg * ac, sb = sg * bc, sL = sg * Lc;
          TC dk[3] = {sL * ck.A * sa, sL * ck.A * sb, sL * ck.B};
          TC x[3];
          mv3(Rc, dk, x);
          x[0] += pc[0];
          x[1] += pc[1];
          x[2] += pc[2];
          int fa;
          const TC viol = marg + ri - poly_sd<TC>(po, jp, x, &fa);
          if (!(viol > TC(0))) continue;
          const T rr = (T)((TC)w.sq_coll * viol);
          const T xf[3] = {(T)x[0], (T)x[1], (T)x[2]};
          const int64_t col = (int64_t)jp * po.F + fa;
          // sd grows along the plane normal: the residual falls along it
          T nvec[3] = {(T)po.pl[col], (T)po.pl[po.ld + col], (T)po.pl[2 * po.ld + col]};
          T row[NZ];
#pragma unroll
          for (int q = 0; q < NZ; ++q) row[q] = T(0);
#pragma unroll
          for (int j = 0; j < NS; ++j) {
            if (j < i) {
              T xmj[3] = {xf[0] - pe[j][0], xf[1] - pe[j][1], xf[2] - pe[j][2]}, c3[3];
              cross3(xmj, nvec, c3);
#pragma unroll
              for (int c = 0; c < NC; ++c)
                row[NC * j + c] = -w.sq_coll * (dot3(W[NC * j + c], c3) + dot3(Pd[NC * j + c], nvec));
            }
          }
          {
            TC nq[3] = {(TC)nvec[0], (TC)nvec[1], (TC)nvec[2]}, q[3];
            mtv3(Rc, nq, q);
            const TC dda[3] = {sL * (ck.A + TC(2) * sa * sa * ck.Ap), sL * TC(2) * sa * sb * ck.Ap, sL * TC(2) * sa * ck.Bp};
            const TC ddb[3] = {sL * TC(2) * sa * sb * ck.Ap, sL * (ck.A + TC(2) * sb * sb * ck.Ap), sL * TC(2) * sb * ck.Bp};
            row[NC * i] = (T)(-(TC)w.sq_coll * sg * dot3(q, dda));
            row[NC * i + 1] = (T)(-(TC)w.sq_coll * sg * dot3(q, ddb));
            if constexpr (EXT) {
              const TC dde[3] = {sg * ck.A * sa, sg * ck.A * sb, sg * ck.B};
              row[NC * i + 2] = (T)(-(TC)w.sq_coll * dot3(q, dde));
            }
          }
          cost += T(0.5) * rr * rr;
#pragma unroll
          for (int k1 = 0; k1 < NZ; ++k1) {
            if (k1 <= NC * i + NC - 1) {
              g[k1] += row[k1] * rr;
#pragma unroll
              for (int k2 = 0; k2 <= k1; ++k2) Hp[tri(k1, k2)] += row[k1] * row[k2];
            }
          }
        }
      }
    }
    ArcCoef<TC> c = arc_coef<TC, true>(s);
    TC Ri[9], di[3];
    seg_R_d(ac, bc, Lc, c, Ri, di);
    {
      TC wa[3] = {-c.C * ac * bc, TC(1) - c.C * bc * bc, -c.A * bc};
      TC wb[3] = {c.C * ac * ac - TC(1), c.C * ac * bc, c.A * ac};
      TC dda[3] = {Lc * (c.A + TC(2) * ac * ac * c.Ap), Lc * TC(2) * ac * bc * c.Ap, Lc * TC(2) * ac * c.Bp};
      TC ddb[3] = {Lc * TC(2) * ac * bc * c.Ap, Lc * (c.A + TC(2) * bc * bc * c.Ap), Lc * TC(2) * bc * c.Bp};
      TC t0[3];
      mv3(Rc, wa, t0);
#pragma unroll
      for (int q = 0; q < 3; ++q) W[NC * i][q] = (T)t0[q];
      mv3(Rc, wb, t0);
#pragma unroll
      for (int q = 0; q < 3; ++q) W[NC * i + 1][q] = (T)t0[q];
      mv3(Rc, dda, t0);
#pragma unroll
      for (int q = 0; q < 3; ++q) Pd[NC * i][q] = (T)t0[q];
      mv3(Rc, ddb, t0);
#pragma unroll
      for (int q = 0; q < 3; ++q) Pd[NC * i + 1][q] = (T)t0[q];
      if constexpr (EXT) {
        const TC dde[3] = {c.A * ac, c.A * bc, c.B};
        mv3(Rc, dde, t0);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          W[NC * i + 2][q] = T(0);
          Pd[NC * i + 2][q] = (T)t0[q];
        }
      }
    }
    TC q[3], Rn[9];
    mv3(Rc, di, q);
    pc[0] += q[0];
    pc[1] += q[1];
    pc[2] += q[2];
    mm3(Rc, Ri, Rn);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = Rn[k];
    pe[i][0] = (T)pc[0];
    pe[i][1] = (T)pc[1];
    pe[i][2] = (T)pc[2];
  }
  T Rt[9], pt[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rt[k] = (T)Rc[k];
  pt[0] = (T)pc[0];
  pt[1] = (T)pc[1];
  pt[2] = (T)pc[2];
  // tip displacement rate of every coordinate (spatial, world frame)
  T dp[NZ][3];
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    const int j = k / NC;
    T rel[3] = {pt[0] - pe[j][0], pt[1] - pe[j][1], pt[2] - pe[j][2]}, c3[3];
    cross3(W[k], rel, c3);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      dp[k][m] = Pd[k][m] + c3[m];
      Jp[m][k] = dp[k][m];
    }
  }
  ptip[0] = pt[0];
  ptip[1] = pt[1];
  ptip[2] = pt[2];
  if (pose) cost += pose_rows<NZ>(w, Rt, pt, W, dp, Tt, Hp, g);
  bounds_normal_eq<NS, NZ, T, EXT>(rb, w, z, 0, Hp, g, cost);
  return cost;
}

// Penalised cost of one configuration against a target pose (eq. 8-10, 17):
// pose, bounds and clearance against M spheres (sphere m, component c at
// sph[m * ms + c * cs], stored as TS).
template <int NS, typename T, typename TS, bool EXT = false, bool SELF = false, bool POLY = false>
CR_HD T cfg_cost(const RobotT<T>& rb, const WeightsT<T>& w, const T* Tt, const T* z, const TS* sph, int M, int64_t ms,
                 int64_t cs, const PolyArgs<TS>& po = PolyArgs<TS>{nullptr, 0, 0, 0}) {
  Fwd<NS, T, EXT> f;
  T c = config_forward<NS, T, false, T, TS, EXT, SELF, POLY>(rb, w, z, sph, M, ms, cs, f, nullptr, po);
  T ft[3], tq[3];
  return c + pose_term<T, false>(w, f.R, f.p, Tt, ft, tq);
}

// lm_ik with clearance rows: the same iteration, the generic per-configuration
// normal equations and cost.
// G > 1 (device only): the G lanes of an aligned lane group carry the same
// configuration and try G step lengths of the line search at once, lane q taking
// 2^-(G r + q) in round r; a ballot over the group takes the first accepted one,
// the sequential search's choice, so the iterates do not depend on G.
template <int NS, typename T, typename TS, bool EXT = false, bool SELF = false, int G = 1, bool POLY = false>
CR_HD void lm_cfg(const RobotT<T>& rb, const WeightsT<T>& w, const T* Tt, T* z, T& lam, int iters, const LMOpts<T>& o,
                  bool& failed, int& trials, const TS* sph, int M, int64_t ms, int64_t cs,
                  const PolyArgs<TS>& po = PolyArgs<TS>{nullptr, 0, 0, 0}) {
  constexpr int NZ = (EXT ? 3 : 2) * NS;
  constexpr int NP = NZ * (NZ + 1) / 2;
  for (int it = 0; it < iters; ++it) {
    T Hp[NP], g[NZ], dl[NZ], ptip[3], Jp[3][NZ];
    const T c0 = local_normal_eq<NS, T, T, TS, EXT, SELF, POLY>(rb, w, z, sph, M, ms, cs, Tt, Hp, g, ptip, Jp, true, po);
    if (!tfinite(c0)) {
      failed = true;
      break;
    }
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      const T hj = Hp[tri(j, j)];
      Hp[tri(j, j)] = hj + lam * (hj > T(1e-12) ? hj : T(1e-12));
      dl[j] = -g[j];
    }
    if (!chol_solve<NZ>(Hp, dl)) {
      if (!(lam < o.lam_max)) break;  // z and lambda would repeat: every later iteration is this one
      lam = lam * T(10) < o.lam_max ? lam * T(10) : o.lam_max;
      continue;
    }
    T gd = T(0);
#pragma unroll
    for (int j = 0; j < NZ; ++j) gd += g[j] * dl[j];
    T alpha = T(1);
    int acc = -1;
    T zt[NZ];
    if constexpr (G == 1) {
      for (int tr = 0; tr < o.ls_max; ++tr) {
#pragma unroll
        for (int j = 0; j < NZ; ++j) zt[j] = z[j] + alpha * dl[j];
        const T c = cfg_cost<NS, T, TS, EXT, SELF, POLY>(rb, w, Tt, zt, sph, M, ms, cs, po);
        ++trials;
        if (c <= c0 + T(1e-4) * alpha * gd) {
          acc = tr;
          break;
        }
        alpha *= T(0.5);
      }
    } else {
#if defined(__HIP_DEVICE_COMPILE__)
      const int lane = threadIdx.x & 63, base = lane & ~(G - 1), q = lane & (G - 1);
      for (int r = 0; r * G < o.ls_max && acc < 0; ++r) {
        const int tr = G * r + q;
        bool ok = false;
        if (tr < o.ls_max) {
          const T at = ldexp(T(1), -tr);
#pragma unroll
          for (int j = 0; j < NZ; ++j) zt[j] = z[j] + at * dl[j];
          const T c = cfg_cost<NS, T, TS, EXT, SELF, POLY>(rb, w, Tt, zt, sph, M, ms, cs, po);
          ok = c <= c0 + T(1e-4) * at * gd;
        }
        ++trials;
        const unsigned grp = (unsigned)((__ballot(ok) >> base) & ((1ull << G) - 1));
        if (grp) acc = G * r + __builtin_ctz(grp);
      }
      if (acc >= 0) {
        alpha = ldexp(T(1), -acc);
#pragma unroll
        for (int j = 0; j < NZ; ++j) zt[j] = z[j] + alpha * dl[j];
      }
#endif
    }
    if (acc >= 0) {
#pragma unroll
      for (int j = 0; j < NZ; ++j) z[j] = zt[j];
      if (acc == 0) lam = lam / T(10) > o.lam_min ? lam / T(10) : o.lam_min;
    } else {
      if (!(lam < o.lam_max)) break;  // rejected at the largest damping: a fixed point of the iteration
      lam = lam * T(10) < o.lam_max ? lam * T(10) : o.lam_max;
    }
  }
}

// True if some backbone point of z lies inside an obstacle sphere inflated by
// its segment's radius (clearance < 0, margin 0); spheres are FP64, sphere m
// component c at sph[c * ld + m].  A sphere whose distance to a segment's arc
// midpoint exceeds L_i / 2 + R + r_i cannot touch the segment.
template <int NS, typename T, bool EXT = false, bool SELF = false, bool POLY = false>
CR_HD bool penetrates(const RobotT<T>& rb, const T* z, const double* sph, int M, int64_t ld,
                      const PolyArgs<double>& po = PolyArgs<double>{nullptr, 0, 0, 0}) {
  constexpr int NC = EXT ? 3 : 2;
  T Rp[9], pp[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rp[k] = (k % 4 == 0) ? T(1) : T(0);
  pp[0] = pp[1] = pp[2] = T(0);
  bool hit = false;
  T Rb[SELF ? NS : 1][9], pb[SELF ? NS : 1][3];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const T a = z[NC * i], b = z[NC * i + 1], s = a * a + b * b;
    const T Li = seg_len<EXT>(rb, z, i), ri = rb.r[i];
    if constexpr (SELF) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Rb[i][k] = Rp[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) pb[i][k] = pp[k];
      // points of segment i against points of every segment m <= i - 2 (margin 0)
#pragma unroll
      for (int m = 0; m < NS; ++m) {
        if (m + 2 > i || hit) continue;
        const T am = z[NC * m], bm = z[NC * m + 1], sm = am * am + bm * bm, Lm = seg_len<EXT>(rb, z, m);
        for (int k = 1; k <= rb.K && !hit; ++k) {
          T q[3];
          seg_point(Rp, pp, a, b, Li, s, T(k) / T(rb.K), q);
          for (int l = 1; l <= rb.K; ++l) {
            T pm[3];
            seg_point(Rb[m], pb[m], am, bm, Lm, sm, T(l) / T(rb.K), pm);
            const T d0 = q[0] - pm[0], d1 = q[1] - pm[1], d2 = q[2] - pm[2];
            if (tsqrt(d0 * d0 + d1 * d1 + d2 * d2) - ri - rb.r[m] < T(0)) hit = true;
          }
        }
      }
    }
    T xm[3];
    seg_point(Rp, pp, a, b, Li, s, T(0.5), xm);
    for (int m = 0; m < M && !hit; ++m) {
      const T cx = (T)sph[m], cy = (T)sph[ld + m], cz = (T)sph[2 * ld + m], rs = (T)sph[3 * ld + m];
      const T e0 = xm[0] - cx, e1 = xm[1] - cy, e2 = xm[2] - cz;
      if (tsqrt(e0 * e0 + e1 * e1 + e2 * e2) - rs - ri - T(0.5) * Li > T(0)) continue;
      for (int k = 1; k <= rb.K; ++k) {
        T x[3];
        seg_point(Rp, pp, a, b, Li, s, T(k) / T(rb.K), x);
        const T d0 = x[0] - cx, d1 = x[1] - cy, d2 = x[2] - cz;
        if (tsqrt(d0 * d0 + d1 * d1 + d2 * d2) - rs - ri < T(0)) hit = true;
      }
    }
    if constexpr (POLY) {
      for (int jp = 0; jp < po.NP && !hit; ++jp) {
        if (poly_sd<T>(po, jp, xm, (int*)nullptr) - ri - T(0.5) * Li > T(0)) continue;
        for (int k = 1; k <= rb.K; ++k) {
          T x[3];
          seg_point(Rp, pp, a, b, Li, s, T(k) / T(rb.K), x);
          if (poly_sd<T>(po, jp, x, (int*)nullptr) - ri < T(0)) hit = true;
        }
      }
    }
    ArcCoef<T> c = arc_coef<T, false>(s);
    T Ri[9], di[3], q[3], Rn[9];
    seg_R_d(a, b, Li, c, Ri, di);
    mv3(Rp, di, q);
    pp[0] += q[0];
    pp[1] += q[1];
    pp[2] += q[2];
    mm3(Rp, Ri, Rn);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rp[k] = Rn[k];
  }
  return hit;
}

// The success test of a configuration against a target pose Tt (3x4 row-major):
// position within 1 mm, rotation within 1 degree, every tendon within its bound
// (1e-6 m), every bending angle within theta_max and no penetration.
template <int NS, typename T>
CR_HD bool ik_success(const RobotT<T>& rb, const T* z, const T* Tt, const double* sph, int M, int64_t ld) {
  T Rc[9], pc[3];
  fk_tip<NS>(rb, z, Rc, pc);
  const T dp[3] = {Tt[3] - pc[0], Tt[7] - pc[1], Tt[11] - pc[2]};
  const T pos = tsqrt(dot3(dp, dp));
  T Re[9], te[3];
  relative_pose(Rc, pc, Tt, Re, te);
  const T v[3] = {T(0.5) * (Re[7] - Re[5]), T(0.5) * (Re[2] - Re[6]), T(0.5) * (Re[3] - Re[1])};
  const T rot = tatan2(tsqrt(dot3(v, v)), T(0.5) * (Re[0] + Re[4] + Re[8] - T(1)));
  if (!(pos <= T(1e-3) && rot <= T(3.14159265358979323846 / 180.0))) return false;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    T u[3];
    ab_to_u(z[2 * i], z[2 * i + 1], rb.r[i], u);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (fabs(u[j]) - rb.umax[i] > T(1e-6)) return false;
    if (tsqrt(z[2 * i] * z[2 * i] + z[2 * i + 1] * z[2 * i + 1]) > rb.theta_max) return false;
  }
  return !(M > 0 && penetrates<NS, T>(rb, z, sph, M, ld));
}

}  // namespace crk
