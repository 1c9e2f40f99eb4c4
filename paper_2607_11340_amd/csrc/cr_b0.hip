// cr_b0.hip -- the plain per-problem FP32 comparison baseline for IK.
//
// Algorithm 1 with the same iteration counts and LM rules as cr_solve_ik, FP32
// throughout (stage 2 included), but built the plain way: one problem at a
// time, a separate kernel per step, residuals and Jacobian by forward-mode dual
// numbers (no hand-derived Jacobian, no adjoint), every intermediate through
// HBM, no fusion of the line search, no graph, no early exit.  Timed against the
// fused solver; not used by it.
#include <float.h>

#include "cr_internal.h"

namespace crk {

// Forward-mode dual number: FP32 value and N directional derivatives.
template <int N>
struct Dual {
  float v, d[N];
  CR_HD Dual() : v(0.0f) {
    for (int k = 0; k < N; ++k) d[k] = 0.0f;
  }
  CR_HD Dual(double x) : v((float)x) {
    for (int k = 0; k < N; ++k) d[k] = 0.0f;
  }
};
template <int N>
CR_HD Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v + b.v;
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N>
CR_HD Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v - b.v;
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N>
CR_HD Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r;
  r.v = -a.v;
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N>
CR_HD Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v * b.v;
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N>
CR_HD Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  const float ib = 1.0f / b.v;
  r.v = a.v * ib;
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
template <int N>
CR_HD Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) {
  a = a + b;
  return a;
}
template <int N>
CR_HD Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) {
  a = a - b;
  return a;
}
template <int N>
CR_HD Dual<N>& operator*=(Dual<N>& a, const Dual<N>& b) {
  a = a * b;
  return a;
}
template <int N>
CR_HD bool operator<(const Dual<N>& a, const Dual<N>& b) { return a.v < b.v; }
template <int N>
CR_HD bool operator>(const Dual<N>& a, const Dual<N>& b) { return a.v > b.v; }
template <int N>
CR_HD bool operator<=(const Dual<N>& a, const Dual<N>& b) { return a.v <= b.v; }
template <int N>
CR_HD bool operator>=(const Dual<N>& a, const Dual<N>& b) { return a.v >= b.v; }
template <int N>
CR_HD bool operator==(const Dual<N>& a, const Dual<N>& b) { return a.v == b.v; }
template <int N>
CR_HD bool operator!=(const Dual<N>& a, const Dual<N>& b) { return a.v != b.v; }
template <int N>
CR_HD Dual<N> fabs(const Dual<N>& a) { return a.v < 0.0f ? -a : a; }

template <int N>
struct Prec<Dual<N>> : Prec<float> {};

template <int N>
CR_HD Dual<N> chain1(const Dual<N>& a, float f, float df) {
  Dual<N> r;
  r.v = f;
  for (int k = 0; k < N; ++k) r.d[k] = df * a.d[k];
  return r;
}
#define CR_DUAL_FUNCS(N)                                                              \
  template <>                                                                         \
  CR_HD Dual<N> tsqrt<Dual<N>>(Dual<N> x) {                                           \
    const float s = sqrtf(x.v);                                                       \
    return chain1(x, s, s > 0.0f ? 0.5f / s : 0.0f);                                  \
  }                                                                                   \
  template <>                                                                         \
  CR_HD Dual<N> tatan2<Dual<N>>(Dual<N> y, Dual<N> x) {                               \
    Dual<N> r;                                                                        \
    r.v = atan2f(y.v, x.v);                                                           \
    const float q = x.v * x.v + y.v * y.v, iq = q > 0.0f ? 1.0f / q : 0.0f;           \
    for (int k = 0; k < N; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) * iq;          \
    return r;                                                                         \
  }                                                                                   \
  template <>                                                                         \
  CR_HD void tsincos<Dual<N>>(Dual<N> x, Dual<N> * s, Dual<N> * c) {                  \
    float sv, cv;                                                                     \
    sincosf(x.v, &sv, &cv);                                                           \
    *s = chain1(x, sv, cv);                                                           \
    *c = chain1(x, cv, -sv);                                                          \
  }                                                                                   \
  template <>                                                                         \
  CR_HD bool tfinite<Dual<N>>(Dual<N> x) {                                            \
    return __builtin_isfinite(x.v);                                                   \
  }
CR_DUAL_FUNCS(2)
CR_DUAL_FUNCS(4)
CR_DUAL_FUNCS(6)
CR_DUAL_FUNCS(8)
CR_DUAL_FUNCS(10)
CR_DUAL_FUNCS(12)
#undef CR_DUAL_FUNCS

template <typename D>
CR_HD RobotT<D> robot_as(const RobotT<float>& rb) {
  RobotT<D> o{};
  o.n = rb.n;
  o.K = rb.K;
  for (int i = 0; i < CR_MAX_SEG; ++i) {
    o.L[i] = D(rb.L[i]);
    o.r[i] = D(rb.r[i]);
    o.umax[i] = D(rb.umax[i]);
    o.Ld[i] = rb.Ld[i];
    o.rd[i] = rb.rd[i];
    o.umaxd[i] = rb.umaxd[i];
  }
  o.theta_max = D(rb.theta_max);
  o.theta_maxd = rb.theta_maxd;
  return o;
}

template <typename D>
CR_HD WeightsT<D> weights_as(const WeightsT<float>& w) {
  WeightsT<D> o{};
  o.w_pos = D(w.w_pos);
  o.w_rot = D(w.w_rot);
  o.sq_lim = D(w.sq_lim);
  o.sq_curv = D(w.sq_curv);
  o.sq_coll = D(w.sq_coll);
  o.margin = D(w.margin);
  o.sq_eq = D(w.sq_eq);
  o.sq_len = D(w.sq_len);
  o.sq_vel = D(w.sq_vel);
  o.sq_acc = D(w.sq_acc);
  o.v_max = D(w.v_max);
  o.a_max = D(w.a_max);
  o.dt = D(w.dt);
  o.has_vmax = w.has_vmax;
  o.has_amax = w.has_amax;
  o.margind = w.margind;
  return o;
}

// Residual vector of the IK cost (eq. 8-9): weighted SE(3) log of T_ee^-1 T,
// then per segment three tendon hinges and the bending hinge.  M = 6 + 4n rows.
template <int NS, typename T>
CR_HD void ik_residuals(const RobotT<T>& rb, const WeightsT<T>& w, const T* Tt, const T* z, T* r) {
  T Rc[9], pc[3], Re[9], te[3], om[3], rho[3], gam, dg;
  fk_tip<NS>(rb, z, Rc, pc);
  relative_pose(Rc, pc, Tt, Re, te);
  log_se3<T, false>(Re, te, om, rho, &gam, &dg);
  for (int k = 0; k < 3; ++k) {
    r[k] = w.w_pos * rho[k];
    r[3 + k] = w.w_rot * om[k];
  }
  for (int i = 0; i < NS; ++i) {
    T ru[3], sg[3], rth;
    bound_residuals<T, T>(rb, w, i, z[2 * i], z[2 * i + 1], ru, sg, &rth);
    for (int j = 0; j < 3; ++j) r[6 + 4 * i + j] = ru[j];
    r[6 + 4 * i + 3] = rth;
  }
}

template <int NS>
__device__ float b0_cost(const RobotT<float>& rb, const WeightsT<float>& w, const float* Tt, const float* z) {
  constexpr int M = 6 + 4 * NS;
  float r[M];
  ik_residuals<NS, float>(rb, w, Tt, z, r);
  float c = 0.0f;
  for (int k = 0; k < M; ++k) c += r[k] * r[k];
  return 0.5f * c;
}

// Per-problem state of the baseline, SoA over the problem's seeds:
// z [NZ][S], zt [NZ][S], lam [S], r [M][S], J [M][NZ][S], Hp [NP][S], g [NZ][S],
// dl [NZ][S], c0, gd, ct [S], flags [S] (bit 0 failed, bit 1 step accepted,
// bit 2 Cholesky failed), acc [S].

template <int NS>
__global__ void k_b0_init(int S, int64_t ld, int64_t col0, const double* __restrict__ useed, RobotT<float> rb,
                          float lam0, float* __restrict__ z, float* __restrict__ lam, int32_t* __restrict__ flags) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  for (int i = 0; i < NS; ++i) {
    float a, b;
    u_to_ab((float)useed[(3 * i) * ld + col0 + s], (float)useed[(3 * i + 1) * ld + col0 + s],
            (float)useed[(3 * i + 2) * ld + col0 + s], rb.r[i], &a, &b);
    z[(2 * i) * S + s] = a;
    z[(2 * i + 1) * S + s] = b;
  }
  lam[s] = lam0;
  flags[s] = 0;
}

// Residuals and Jacobian by forward-mode dual numbers; cost at z.
template <int NS>
__global__ void k_b0_resjac(int S, RobotT<float> rb, WeightsT<float> w, const float* __restrict__ Tt,
                            const float* __restrict__ z, float* __restrict__ r, float* __restrict__ J,
                            float* __restrict__ c0, int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS, M = 6 + 4 * NS;
  using D = Dual<NZ>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 1)) return;
  const RobotT<D> rd = robot_as<D>(rb);
  const WeightsT<D> wd = weights_as<D>(w);
  D zd[NZ], Td[12], rr[M];
  for (int k = 0; k < NZ; ++k) {
    zd[k] = D(z[k * S + s]);
    zd[k].d[k] = 1.0f;
  }
  for (int k = 0; k < 12; ++k) Td[k] = D(Tt[k]);
  ik_residuals<NS, D>(rd, wd, Td, zd, rr);
  float c = 0.0f;
  for (int m = 0; m < M; ++m) {
    r[m * S + s] = rr[m].v;
    c += rr[m].v * rr[m].v;
    for (int k = 0; k < NZ; ++k) J[(m * NZ + k) * S + s] = rr[m].d[k];
  }
  c0[s] = 0.5f * c;
  if (!tfinite(c)) flags[s] |= 1;
}

template <int NS>
__global__ void k_b0_normal(int S, const float* __restrict__ r, const float* __restrict__ J, float* __restrict__ Hp,
                            float* __restrict__ g, const int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS, M = 6 + 4 * NS;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 1)) return;
  for (int a = 0; a < NZ; ++a) {
    float ga = 0.0f;
    for (int m = 0; m < M; ++m) ga += J[(m * NZ + a) * S + s] * r[m * S + s];
    g[a * S + s] = ga;
    for (int b = 0; b <= a; ++b) {
      float h = 0.0f;
      for (int m = 0; m < M; ++m) h += J[(m * NZ + a) * S + s] * J[(m * NZ + b) * S + s];
      Hp[tri(a, b) * S + s] = h;
    }
  }
}

// Damped Cholesky step (H + lambda D) delta = -g and g.delta.
template <int NS>
__global__ void k_b0_step(int S, const float* __restrict__ Hp, const float* __restrict__ g,
                          const float* __restrict__ lam, float* __restrict__ dl, float* __restrict__ gd,
                          int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS, NP = NZ * (NZ + 1) / 2;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 1)) return;
  float A[NP], x[NZ];
  for (int k = 0; k < NP; ++k) A[k] = Hp[k * S + s];
  for (int j = 0; j < NZ; ++j) {
    const float hj = A[tri(j, j)];
    A[tri(j, j)] = hj + lam[s] * (hj > 1e-12f ? hj : 1e-12f);
    x[j] = -g[j * S + s];
  }
  const bool ok = chol_solve<NZ>(A, x);
  float d = 0.0f;
  for (int j = 0; j < NZ; ++j) {
    dl[j * S + s] = x[j];
    d += g[j * S + s] * x[j];
  }
  gd[s] = d;
  flags[s] = (flags[s] & 1) | (ok ? 0 : 4);
}

// One line-search trial: cost at z + alpha delta for seeds without an accepted step.
template <int NS>
__global__ void k_b0_trial(int S, RobotT<float> rb, WeightsT<float> w, const float* __restrict__ Tt, float alpha,
                           const float* __restrict__ z, const float* __restrict__ dl, float* __restrict__ zt,
                           float* __restrict__ ct, const int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 7)) return;
  float tt[12], zz[NZ];
  for (int k = 0; k < 12; ++k) tt[k] = Tt[k];
  for (int k = 0; k < NZ; ++k) {
    zz[k] = z[k * S + s] + alpha * dl[k * S + s];
    zt[k * S + s] = zz[k];
  }
  ct[s] = b0_cost<NS>(rb, w, tt, zz);
}

// Armijo test of the trial; an accepted trial is copied into z.
template <int NS>
__global__ void k_b0_accept(int S, int trial, float alpha, const float* __restrict__ c0, const float* __restrict__ gd,
                            const float* __restrict__ ct, const float* __restrict__ zt, float* __restrict__ z,
                            int32_t* __restrict__ acc, int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 7)) return;
  if (ct[s] <= c0[s] + 1e-4f * alpha * gd[s]) {
    for (int k = 0; k < NZ; ++k) z[k * S + s] = zt[k * S + s];
    acc[s] = trial;
    flags[s] |= 2;
  }
}

// Damping update after the trials.
__global__ void k_b0_lambda(int S, float lam_min, float lam_max, float* __restrict__ lam, int32_t* __restrict__ acc,
                            int32_t* __restrict__ flags) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 1)) return;
  float l = lam[s];
  if ((flags[s] & 2) && acc[s] == 0) l = l / 10.0f > lam_min ? l / 10.0f : lam_min;
  if (!(flags[s] & 2)) l = l * 10.0f < lam_max ? l * 10.0f : lam_max;
  lam[s] = l;
  flags[s] &= 1;
  acc[s] = -1;
}

// SelectTop keys and final cost at the end of a stage.
template <int NS>
__global__ void k_b0_keys(int S, RobotT<float> rb, WeightsT<float> w, const float* __restrict__ Tt,
                          const float* __restrict__ z, float* __restrict__ e, float* __restrict__ pen,
                          float* __restrict__ cost, int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  float tt[12], zz[NZ];
  for (int k = 0; k < 12; ++k) tt[k] = Tt[k];
  for (int k = 0; k < NZ; ++k) zz[k] = z[k * S + s];
  float ee;
  const float c = ik_cost<NS>(rb, w, tt, zz, &ee);
  e[s] = ee;
  pen[s] = 0.0f;
  cost[s] = c;
  if (!tfinite(c) || !tfinite(ee)) flags[s] |= 1;
}

// Stage-2 start: the kept candidates' z, fresh damping.
template <int NS>
__global__ void k_b0_gather(int S, int nf, const float* __restrict__ z1, const int32_t* __restrict__ sel,
                            float lam0, float* __restrict__ z2, float* __restrict__ lam, int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nf) return;
  const int s = sel[k];
  for (int m = 0; m < NZ; ++m) z2[m * nf + k] = s >= 0 ? z1[m * S + s] : 0.0f;
  lam[k] = lam0;
  flags[k] = s >= 0 ? 0 : 1;
}

__global__ void k_b0_fill(int n, int32_t* __restrict__ x, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_b0_target(const double* __restrict__ T, int64_t P, int64_t p, float* __restrict__ Tt) {
  const int c = threadIdx.x;
  if (c < 12) Tt[c] = (float)T[c * P + p];
}

// Argmin over the candidates (ties to the lower seed) and the FP64 assessment.
template <int NS>
__global__ void k_b0_finalize(RobotT<double> rb, int nc, const int32_t* __restrict__ sel, const float* __restrict__ zc,
                              const float* __restrict__ costc, const int32_t* __restrict__ flagc,
                              const double* __restrict__ T, int64_t P, int64_t p, const double* __restrict__ sph,
                              int64_t sph_off, int64_t sph_ld, int M, double* __restrict__ u_out,
                              double* __restrict__ err_out, int32_t* __restrict__ status_out) {
  constexpr int NZ = 2 * NS;
  if (threadIdx.x != 0) return;
  int best = -1, best_seed = 0;
  float bc = 0.0f;
  for (int k = 0; k < nc; ++k) {
    const int seed = sel ? sel[k] : k;
    if (seed < 0 || (flagc[k] & 1) || !tfinite(costc[k])) continue;
    if (best < 0 || costc[k] < bc || (costc[k] == bc && seed < best_seed)) {
      best = k;
      bc = costc[k];
      best_seed = seed;
    }
  }
  if (best < 0) {
    for (int m = 0; m < 3 * NS; ++m) u_out[m * P + p] = __builtin_nan("");
    err_out[p] = err_out[P + p] = __builtin_nan("");
    status_out[p] = CR_NONFINITE;
    return;
  }
  double z[NZ], tt[12];
  for (int m = 0; m < NZ; ++m) z[m] = (double)zc[m * nc + best];
  for (int c = 0; c < 12; ++c) tt[c] = T[c * P + p];
  double Rc[9], pc[3], Re[9], te[3];
  fk_tip<NS>(rb, z, Rc, pc);
  const double dp[3] = {tt[3] - pc[0], tt[7] - pc[1], tt[11] - pc[2]};
  const double pos = sqrt(dot3(dp, dp));
  relative_pose(Rc, pc, tt, Re, te);
  const double v[3] = {0.5 * (Re[7] - Re[5]), 0.5 * (Re[2] - Re[6]), 0.5 * (Re[3] - Re[1])};
  const double rot = atan2(sqrt(dot3(v, v)), 0.5 * (Re[0] + Re[4] + Re[8] - 1.0));
  double viol = -DBL_MAX, thx = -DBL_MAX;
  for (int i = 0; i < NS; ++i) {
    double u[3];
    ab_to_u(z[2 * i], z[2 * i + 1], rb.rd[i], u);
    for (int j = 0; j < 3; ++j) {
      u_out[(3 * i + j) * P + p] = u[j];
      viol = fmax(viol, ::fabs(u[j]) - rb.umaxd[i]);
    }
    thx = fmax(thx, sqrt(z[2 * i] * z[2 * i] + z[2 * i + 1] * z[2 * i + 1]) - rb.theta_maxd);
  }
  int32_t st = 0;
  if (viol > 1e-6 || thx > 0.0) st |= CR_LIMIT_VIOLATION;
  if (!(pos <= 1e-3 && rot <= 3.14159265358979323846 / 180.0)) st |= CR_NOT_CONVERGED;
  if (M > 0 && penetrates<NS, double>(rb, z, sph + sph_off, M, sph_ld)) st |= CR_COLLISION;
  err_out[p] = pos;
  err_out[P + p] = rot;
  status_out[p] = st == 0 ? CR_SOLVED : st;
}

// Cost rows of one waypoint configuration that involve it alone, in type D (float,
// or a dual number carrying d/dz): pose (paths), bounds, clearance.  Calls
// row(r, is_clearance) for every row; returns the lifts u [3n] and the tip position.
template <int NS, typename D, typename F>
__device__ void b0t_rows(const RobotT<D>& rb, const WeightsT<D>& w, int kind, const float* Tt, const double* sph,
                         int64_t sph_off, int64_t sph_ld, int M, const D* z, D* u, D* ptip, F row) {
  D Rc[9], pc[3];
  for (int k = 0; k < 9; ++k) Rc[k] = D((k % 4 == 0) ? 1.0 : 0.0);
  pc[0] = pc[1] = pc[2] = D(0.0);
  const int K = rb.K;
  for (int i = 0; i < NS; ++i) {
    const D a = z[2 * i], b = z[2 * i + 1], s = a * a + b * b;
    for (int k = 1; k <= K && M > 0; ++k) {
      D x[3];
      seg_point(Rc, pc, a, b, rb.L[i], s, D((double)k / (double)K), x);
      for (int m = 0; m < M; ++m) {
        const float cx = (float)sph[sph_off + m], cy = (float)sph[sph_off + sph_ld + m];
        const float cz = (float)sph[sph_off + 2 * sph_ld + m], rs = (float)sph[sph_off + 3 * sph_ld + m];
        const float reach = rs + (float)rb.rd[i] + (float)w.margind;
        const D d0 = x[0] - D(cx), d1 = x[1] - D(cy), d2 = x[2] - D(cz);
        const D dist = tsqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const D viol = D(reach) - dist;
        if (viol > D(0.0)) row(w.sq_coll * viol, true);
      }
    }
    ArcCoef<D> c = arc_coef<D, false>(s);
    D Ri[9], di[3], q[3], Rn[9];
    seg_R_d(a, b, rb.L[i], c, Ri, di);
    mv3(Rc, di, q);
    for (int k = 0; k < 3; ++k) pc[k] += q[k];
    mm3(Rc, Ri, Rn);
    for (int k = 0; k < 9; ++k) Rc[k] = Rn[k];
    ab_to_u(a, b, rb.r[i], u + 3 * i);
    D ru[3], sg[3], rth;
    bound_residuals<D, D>(rb, w, i, a, b, ru, sg, &rth);
    for (int k = 0; k < 3; ++k) row(ru[k], false);
    row(rth, false);
  }
  for (int k = 0; k < 3; ++k) ptip[k] = pc[k];
  if (kind == CR_KIND_PATH) {
    D Td[12], Re[9], te[3], om[3], rho[3], gam, dg;
    for (int k = 0; k < 12; ++k) Td[k] = D(Tt[k]);
    relative_pose(Rc, pc, Td, Re, te);
    log_se3<D, false>(Re, te, om, rho, &gam, &dg);
    for (int k = 0; k < 3; ++k) {
      row(w.w_pos * rho[k], false);
      row(w.w_rot * om[k], false);
    }
  }
}

// IK among spheres: the clearance rows vary in number (the active point-sphere
// pairs), so J^T J and J^T r are accumulated as the dual-number rows are formed
// (pose, bounds, clearance), and the cost with them.
template <int NS>
__global__ void k_b0_normal_sph(int S, RobotT<float> rb, WeightsT<float> w, const float* __restrict__ Tt,
                                const double* __restrict__ sph, int64_t sph_off, int64_t sph_ld, int M,
                                const float* __restrict__ z, float* __restrict__ Hp, float* __restrict__ g,
                                float* __restrict__ c0, int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS, NU = 3 * NS, NP = NZ * (NZ + 1) / 2;
  using D = Dual<NZ>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 1)) return;
  const RobotT<D> rd = robot_as<D>(rb);
  const WeightsT<D> wd = weights_as<D>(w);
  D zd[NZ], u[NU], pt[3];
  for (int k = 0; k < NZ; ++k) {
    zd[k] = D(z[k * S + s]);
    zd[k].d[k] = 1.0f;
  }
  float tt[12];
  for (int k = 0; k < 12; ++k) tt[k] = Tt[k];
  float H[NP], gg[NZ], c = 0.0f;
  for (int k = 0; k < NP; ++k) H[k] = 0.0f;
  for (int k = 0; k < NZ; ++k) gg[k] = 0.0f;
  b0t_rows<NS, D>(rd, wd, CR_KIND_PATH, tt, sph, sph_off, sph_ld, M, zd, u, pt, [&](const D& r, bool) {
    c += 0.5f * r.v * r.v;
    for (int a = 0; a < NZ; ++a) {
      gg[a] += r.d[a] * r.v;
      for (int b = 0; b <= a; ++b) H[tri(a, b)] += r.d[a] * r.d[b];
    }
  });
  for (int k = 0; k < NP; ++k) Hp[k * S + s] = H[k];
  for (int k = 0; k < NZ; ++k) g[k * S + s] = gg[k];
  c0[s] = c;
  if (!tfinite(c)) flags[s] |= 1;
}

// FP32 cost of the IK rows among spheres at z (pen: the clearance part).
template <int NS>
__device__ float b0_cost_sph(const RobotT<float>& rb, const WeightsT<float>& w, const float* tt, const double* sph,
                             int64_t sph_off, int64_t sph_ld, int M, const float* z, float* pen) {
  float u[3 * NS], pt[3], c = 0.0f, cp = 0.0f;
  b0t_rows<NS, float>(rb, w, CR_KIND_PATH, tt, sph, sph_off, sph_ld, M, z, u, pt, [&](float r, bool coll) {
    c += 0.5f * r * r;
    if (coll) cp += 0.5f * r * r;
  });
  if (pen) *pen = cp;
  return c;
}

template <int NS>
__global__ void k_b0_trial_sph(int S, RobotT<float> rb, WeightsT<float> w, const float* __restrict__ Tt,
                               const double* __restrict__ sph, int64_t sph_off, int64_t sph_ld, int M, float alpha,
                               const float* __restrict__ z, const float* __restrict__ dl, float* __restrict__ zt,
                               float* __restrict__ ct, const int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 7)) return;
  float tt[12], zz[NZ];
  for (int k = 0; k < 12; ++k) tt[k] = Tt[k];
  for (int k = 0; k < NZ; ++k) {
    zz[k] = z[k * S + s] + alpha * dl[k * S + s];
    zt[k * S + s] = zz[k];
  }
  ct[s] = b0_cost_sph<NS>(rb, w, tt, sph, sph_off, sph_ld, M, zz, nullptr);
}

// SelectTop keys among spheres: pose error, clearance penalty, cost.
template <int NS>
__global__ void k_b0_keys_sph(int S, RobotT<float> rb, WeightsT<float> w, const float* __restrict__ Tt,
                              const double* __restrict__ sph, int64_t sph_off, int64_t sph_ld, int M,
                              const float* __restrict__ z, float* __restrict__ e, float* __restrict__ pen,
                              float* __restrict__ cost, int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  float tt[12], zz[NZ];
  for (int k = 0; k < 12; ++k) tt[k] = Tt[k];
  for (int k = 0; k < NZ; ++k) zz[k] = z[k * S + s];
  float ee, pn;
  (void)ik_cost<NS>(rb, w, tt, zz, &ee);
  const float c = b0_cost_sph<NS>(rb, w, tt, sph, sph_off, sph_ld, M, zz, &pn);
  e[s] = ee;
  pen[s] = pn;
  cost[s] = c;
  if (!tfinite(c) || !tfinite(ee)) flags[s] |= 1;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct B0Ws {
  float *z, *zt, *lam, *r, *J, *Hp, *g, *dl, *c0, *gd, *ct, *e, *pen, *cost, *z2, *Tt;
  int32_t *flags, *acc, *sel;
};

static size_t b0_layout(int ns, int S, int nf, char* base, B0Ws* w) {
  const int NZ = 2 * ns, M = 6 + 4 * ns, NP = NZ * (NZ + 1) / 2;
  const int Sx = S > nf ? S : nf;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t at = off;
    off += (b + 255) & ~(size_t)255;
    return base ? (void*)(base + at) : nullptr;
  };
  B0Ws x{};
  x.z = (float*)take(4 * (size_t)NZ * Sx);
  x.zt = (float*)take(4 * (size_t)NZ * Sx);
  x.lam = (float*)take(4 * (size_t)Sx);
  x.r = (float*)take(4 * (size_t)M * Sx);
  x.J = (float*)take(4 * (size_t)M * NZ * Sx);
  x.Hp = (float*)take(4 * (size_t)NP * Sx);
  x.g = (float*)take(4 * (size_t)NZ * Sx);
  x.dl = (float*)take(4 * (size_t)NZ * Sx);
  x.c0 = (float*)take(4 * (size_t)Sx);
  x.gd = (float*)take(4 * (size_t)Sx);
  x.ct = (float*)take(4 * (size_t)Sx);
  x.e = (float*)take(4 * (size_t)Sx);
  x.pen = (float*)take(4 * (size_t)Sx);
  x.cost = (float*)take(4 * (size_t)Sx);
  x.z2 = (float*)take(4 * (size_t)NZ * Sx);
  x.Tt = (float*)take(4 * 12);
  x.flags = (int32_t*)take(4 * (size_t)Sx);
  x.acc = (int32_t*)take(4 * (size_t)Sx);
  x.sel = (int32_t*)take(4 * (size_t)(nf > 0 ? nf : 1));
  if (w) *w = x;
  return off;
}

size_t b0_workspace_bytes(const cr_robot& rb, int S, const cr_opts& o) {
  return b0_layout(rb.n_seg, S, o.n_final, nullptr, nullptr);
}

// Spheres of the problem being solved (M = 0: none).
struct B0Sph {
  const double* sph;
  int64_t off, ld;
  int M;
};

template <int NS>
static cr_status b0_stage(const RobotT<float>& rb, const WeightsT<float>& w, const cr_opts& o, int S, int iters,
                          const B0Ws& ws, float* z, const B0Sph& sp, hipStream_t st) {
  const dim3 grid((S + 63) / 64), blk(64);
  for (int it = 0; it < iters; ++it) {
    if (sp.M > 0) {
      hipLaunchKernelGGL((k_b0_normal_sph<NS>), grid, blk, 0, st, S, rb, w, ws.Tt, sp.sph, sp.off, sp.ld, sp.M, z,
                         ws.Hp, ws.g, ws.c0, ws.flags);
    } else {
      hipLaunchKernelGGL((k_b0_resjac<NS>), grid, blk, 0, st, S, rb, w, ws.Tt, z, ws.r, ws.J, ws.c0, ws.flags);
      hipLaunchKernelGGL((k_b0_normal<NS>), grid, blk, 0, st, S, ws.r, ws.J, ws.Hp, ws.g, ws.flags);
    }
    hipLaunchKernelGGL((k_b0_step<NS>), grid, blk, 0, st, S, ws.Hp, ws.g, ws.lam, ws.dl, ws.gd, ws.flags);
    float alpha = 1.0f;
    for (int tr = 0; tr < o.ls_max; ++tr) {
      if (sp.M > 0)
        hipLaunchKernelGGL((k_b0_trial_sph<NS>), grid, blk, 0, st, S, rb, w, ws.Tt, sp.sph, sp.off, sp.ld, sp.M,
                           alpha, z, ws.dl, ws.zt, ws.ct, ws.flags);
      else
        hipLaunchKernelGGL((k_b0_trial<NS>), grid, blk, 0, st, S, rb, w, ws.Tt, alpha, z, ws.dl, ws.zt, ws.ct,
                           ws.flags);
      hipLaunchKernelGGL((k_b0_accept<NS>), grid, blk, 0, st, S, tr, alpha, ws.c0, ws.gd, ws.ct, ws.zt, z, ws.acc,
                         ws.flags);
      alpha *= 0.5f;
    }
    hipLaunchKernelGGL(k_b0_lambda, grid, blk, 0, st, S, (float)o.lambda_min, (float)o.lambda_max, ws.lam, ws.acc,
                       ws.flags);
  }
  return check_hip(hipGetLastError(), "baseline stage");
}

template <int NS>
static cr_status b0_run(const cr_robot& rb0, const cr_spheres* spheres, int64_t P, const double* T, int S,
                        const double* useed, const cr_weights& w0, const cr_opts& o, double* u_out, double* err_out,
                        int32_t* status_out, const B0Ws& ws, hipStream_t st) {
  const RobotT<float> rb = robot_to<float>(rb0);
  const WeightsT<float> w = weights_to<float>(w0);
  const RobotT<double> rbd = robot_to<double>(rb0);
  const dim3 grid((S + 63) / 64), blk(64);
  const int nf = o.n_final;
  cr_status rc = CR_OK;
  for (int64_t p = 0; p < P && rc == CR_OK; ++p) {
    B0Sph sp{nullptr, 0, 0, 0};
    if (spheres && spheres->n_sph > 0)
      sp = B0Sph{(const double*)spheres->sph, spheres->per_problem ? p * spheres->n_sph : 0, spheres->ld,
                 spheres->n_sph};
    hipLaunchKernelGGL(k_b0_target, dim3(1), dim3(64), 0, st, T, P, p, ws.Tt);
    hipLaunchKernelGGL((k_b0_init<NS>), grid, blk, 0, st, S, P * (int64_t)S, p * (int64_t)S, useed, rb,
                       (float)o.lambda0, ws.z, ws.lam, ws.flags);
    hipLaunchKernelGGL(k_b0_fill, grid, blk, 0, st, S, ws.acc, -1);
    rc = b0_stage<NS>(rb, w, o, S, o.k_init, ws, ws.z, sp, st);
    if (rc != CR_OK) break;
    if (sp.M > 0)
      hipLaunchKernelGGL((k_b0_keys_sph<NS>), grid, blk, 0, st, S, rb, w, ws.Tt, sp.sph, sp.off, sp.ld, sp.M, ws.z,
                         ws.e, ws.pen, ws.cost, ws.flags);
    else
      hipLaunchKernelGGL((k_b0_keys<NS>), grid, blk, 0, st, S, rb, w, ws.Tt, ws.z, ws.e, ws.pen, ws.cost, ws.flags);
    if (nf > 0) {
      rc = launch_select(1, S, 2 * NS, ws.z, ws.e, ws.pen, ws.flags, nf, o.dup_eps, ws.sel, CR_F32, st);
      if (rc != CR_OK) break;
      const dim3 g2((nf + 63) / 64);
      hipLaunchKernelGGL((k_b0_gather<NS>), g2, blk, 0, st, S, nf, ws.z, ws.sel, (float)o.lambda0, ws.z2, ws.lam,
                         ws.flags);
      hipLaunchKernelGGL(k_b0_fill, g2, blk, 0, st, nf, ws.acc, -1);
      rc = b0_stage<NS>(rb, w, o, nf, o.k_final, ws, ws.z2, sp, st);
      if (rc != CR_OK) break;
      if (sp.M > 0)
        hipLaunchKernelGGL((k_b0_keys_sph<NS>), g2, blk, 0, st, nf, rb, w, ws.Tt, sp.sph, sp.off, sp.ld, sp.M, ws.z2,
                           ws.e, ws.pen, ws.cost, ws.flags);
      else
        hipLaunchKernelGGL((k_b0_keys<NS>), g2, blk, 0, st, nf, rb, w, ws.Tt, ws.z2, ws.e, ws.pen, ws.cost,
                           ws.flags);
      hipLaunchKernelGGL((k_b0_finalize<NS>), dim3(1), dim3(64), 0, st, rbd, nf, ws.sel, ws.z2, ws.cost, ws.flags, T,
                         P, p, sp.sph, sp.off, sp.ld, sp.M, u_out, err_out, status_out);
    } else {
      hipLaunchKernelGGL((k_b0_finalize<NS>), dim3(1), dim3(64), 0, st, rbd, S, (const int32_t*)nullptr, ws.z,
                         ws.cost, ws.flags, T, P, p, sp.sph, sp.off, sp.ld, sp.M, u_out, err_out, status_out);
    }
    rc = check_hip(hipGetLastError(), "baseline solve");
  }
  return rc;
}

cr_status launch_b0_ik(const cr_robot& rb, const cr_spheres* sp, int64_t P, const double* T, int S,
                       const double* useed, const cr_weights& w, const cr_opts& o, double* u_out, double* err_out,
                       int32_t* status_out, void* wsmem, hipStream_t st) {
  B0Ws ws;
  b0_layout(rb.n_seg, S, o.n_final, (char*)wsmem, &ws);
#define CR_B0_CASE(N) \
  case N:             \
    return b0_run<N>(rb, sp, P, T, S, useed, w, o, u_out, err_out, status_out, ws, st);
  switch (rb.n_seg) {
    CR_B0_CASE(1)
    CR_B0_CASE(2)
    CR_B0_CASE(3)
    CR_B0_CASE(4)
    CR_B0_CASE(5)
    CR_B0_CASE(6)
    default:
      return fail(CR_EINVAL, "n_seg out of range");
  }
#undef CR_B0_CASE
}


// ===========================================================================
// Paths and trajectories (eq. 11-17), the same plain way: one problem at a time
// (its S trajectories), FP32 throughout, a separate kernel per step, every
// intermediate through HBM, no graph, no early exit.  Each waypoint's own rows
// (pose for paths, bounds, clearance against every sphere and backbone point,
// no culls) get their Jacobian by forward-mode dual numbers; the coupling rows
// (tendon velocity and acceleration, tip path length, endpoints) are linear in
// the lifts and the tip positions, whose derivatives the same dual pass
// records.  The block-pentadiagonal normal equations are factored by one
// thread per trajectory walking its records in HBM.
// Layouts, waypoint configuration j = s * Tn + t of the problem's trajectory s:
// Z [j][NZ], records [j][Rec], U [j][3n], dU [j][3n][NZ], Pt [j][3], dP [j][3][NZ],
// cw / pw [j] (waypoint cost and clearance part), per trajectory c0, gd, ct, lam,
// flags (bit 0 failed, 1 step accepted, 2 factorisation failed), acc.
// ===========================================================================

template <int NS>
struct B0Rec {
  static constexpr int NZ = 2 * NS;
  static constexpr int OH = 0, OB = NZ * NZ, OC = 2 * NZ * NZ, OG = 3 * NZ * NZ, OY = OG + NZ;
  static constexpr int SIZE = OY + NZ;
};

// Problem q's row of the baseline's table: global task, seed, output and sphere
// offsets, candidates local to the problem (first trajectory 0).
__global__ void k_b0t_row(int kind, int64_t P, int64_t q, int S, int Tn, int M, int per_problem, int64_t sph_ld,
                          TrajProb* __restrict__ row) {
  if (threadIdx.x != 0) return;
  TrajProb r;
  r.Tn = Tn;
  r.S = S;
  r.M = M;
  r.idx = (int32_t)q;
  r.traj0 = 0;
  r.wp0 = 0;
  r.tn0 = 0;
  r.task = kind == CR_KIND_PATH ? q * Tn : q;
  r.task_ld = kind == CR_KIND_PATH ? P * Tn : P;
  r.seed = q * S * (int64_t)Tn;
  r.seed_ld = P * S * (int64_t)Tn;
  r.out = q * Tn;
  r.out_ld = P * Tn;
  r.sph = per_problem ? q * M : 0;
  r.sph_ld = sph_ld;
  *row = r;
}

template <int NS>
__global__ void k_b0t_init(const TrajProb* __restrict__ row, const double* __restrict__ useed, RobotT<float> rb,
                           float lam0, float* __restrict__ Z, float* __restrict__ lam, int32_t* __restrict__ flags,
                           int32_t* __restrict__ acc) {
  constexpr int NZ = 2 * NS;
  const TrajProb pr = *row;
  const int N = pr.S * pr.Tn;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  for (int i = 0; i < NS; ++i)
    u_to_ab((float)useed[pr.seed + (3 * i) * pr.seed_ld + j], (float)useed[pr.seed + (3 * i + 1) * pr.seed_ld + j],
            (float)useed[pr.seed + (3 * i + 2) * pr.seed_ld + j], rb.r[i], &Z[j * NZ + 2 * i], &Z[j * NZ + 2 * i + 1]);
  if (j < pr.S) {
    lam[j] = lam0;
    flags[j] = 0;
    acc[j] = -1;
  }
}

// Reference pose of waypoint t (paths), 12 values.
__device__ inline void b0t_pose(const TrajProb& pr, const double* task, int t, float* Tt) {
  for (int c = 0; c < 12; ++c) Tt[c] = (float)task[pr.task + c * pr.task_ld + t];
}

// Each waypoint's own rows by forward-mode dual numbers: H_tt, g_t, its cost, and
// the lifts and tip position with their derivatives.
template <int NS>
__global__ void k_b0t_local(const TrajProb* __restrict__ row, int S, int kind, RobotT<float> rb, WeightsT<float> w,
                            const double* __restrict__ task, const double* __restrict__ sph,
                            const float* __restrict__ Z, float* __restrict__ blk, float* __restrict__ U,
                            float* __restrict__ dU, float* __restrict__ Pt, float* __restrict__ dP,
                            float* __restrict__ cw, const int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS, NU = 3 * NS, NP = NZ * (NZ + 1) / 2;
  using D = Dual<NZ>;
  using R = B0Rec<NS>;
  const TrajProb pr = *row;
  const int Tn = pr.Tn, N = S * Tn;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N || (flags[j / Tn] & 1)) return;
  const int t = j - (j / Tn) * Tn;
  const RobotT<D> rd = robot_as<D>(rb);
  const WeightsT<D> wd = weights_as<D>(w);
  D z[NZ], u[NU], pt[3];
  for (int k = 0; k < NZ; ++k) {
    z[k] = D(Z[j * NZ + k]);
    z[k].d[k] = 1.0f;
  }
  float Tt[12] = {0};
  if (kind == CR_KIND_PATH) b0t_pose(pr, task, t, Tt);
  float H[NP], g[NZ], c = 0.0f;
  for (int k = 0; k < NP; ++k) H[k] = 0.0f;
  for (int k = 0; k < NZ; ++k) g[k] = 0.0f;
  b0t_rows<NS, D>(rd, wd, kind, Tt, sph, pr.sph, pr.sph_ld, pr.M, z, u, pt, [&](const D& r, bool) {
    c += 0.5f * r.v * r.v;
    for (int a = 0; a < NZ; ++a) {
      g[a] += r.d[a] * r.v;
      for (int b = 0; b <= a; ++b) H[tri(a, b)] += r.d[a] * r.d[b];
    }
  });
  float* rec = blk + (int64_t)j * R::SIZE;
  for (int a = 0; a < NZ; ++a) {
    for (int b = 0; b < NZ; ++b) rec[R::OH + b * NZ + a] = a >= b ? H[tri(a, b)] : H[tri(b, a)];
    rec[R::OG + a] = g[a];
  }
  for (int m = 0; m < NU; ++m) {
    U[j * NU + m] = u[m].v;
    for (int k = 0; k < NZ; ++k) dU[(j * NU + m) * NZ + k] = u[m].d[k];
  }
  for (int c3 = 0; c3 < 3; ++c3) {
    Pt[j * 3 + c3] = pt[c3].v;
    for (int k = 0; k < NZ; ++k) dP[(j * 3 + c3) * NZ + k] = pt[c3].d[k];
  }
  cw[j] = c;
}

// Bending coordinates of the start (end 0) or goal (end 1) of a trajectory problem.
template <int NS>
__device__ inline void b0t_end(const TrajProb& pr, const double* task, const RobotT<float>& rb, int end, float* ze) {
  for (int i = 0; i < NS; ++i) {
    const double* u = task + pr.task + (int64_t)(end * 3 * NS + 3 * i) * pr.task_ld;
    u_to_ab((float)u[0], (float)u[pr.task_ld], (float)u[2 * pr.task_ld], rb.r[i], &ze[2 * i], &ze[2 * i + 1]);
  }
}

// Coupling rows that involve waypoint t: tendon velocity rows centred at t and
// t + 1, acceleration rows centred at t .. t + 2 (with their hinges), tip path
// length rows centred at t and t + 1, endpoint rows.  Adds to H_tt and g_t,
// writes H_{t,t-1} and H_{t,t-2}; the cost of the rows centred at t goes to cw.
template <int NS>
__global__ void k_b0t_couple(const TrajProb* __restrict__ row, int S, int kind, RobotT<float> rb, WeightsT<float> w,
                             const double* __restrict__ task, const float* __restrict__ Z, float* __restrict__ blk,
                             const float* __restrict__ U, const float* __restrict__ dU, const float* __restrict__ Pt,
                             const float* __restrict__ dP, float* __restrict__ cw, const int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS, NU = 3 * NS;
  using R = B0Rec<NS>;
  const TrajProb pr = *row;
  const int Tn = pr.Tn, H = Tn - 1, N = S * Tn;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N || (flags[j / Tn] & 1)) return;
  const int t = j - (j / Tn) * Tn;
  float* rec = blk + (int64_t)j * R::SIZE;
  float Hs[NZ][NZ], Bk[NZ][NZ], Ck[NZ][NZ], g[NZ];
  for (int a = 0; a < NZ; ++a) {
    g[a] = rec[R::OG + a];
    for (int b = 0; b < NZ; ++b) {
      Hs[a][b] = rec[R::OH + b * NZ + a];
      Bk[a][b] = Ck[a][b] = 0.0f;
    }
  }
  float c = 0.0f;
  const float idt = 1.0f / w.dt, idt2 = idt * idt;
  // adds coefficient-weighted outer products of derivative rows: X += ca cb da db^T
  auto outer = [&](float (*X)[NZ], float ca, const float* da, float cb, const float* db) {
    for (int a = 0; a < NZ; ++a)
      for (int b = 0; b < NZ; ++b) X[a][b] += ca * cb * da[a] * db[b];
  };
  for (int m = 0; m < NU; ++m) {
    // velocity rows v(tau) = (u(tau) - u(tau - 1)) / dt, tau = t, t + 1
    for (int k = 0; k < 2; ++k) {
      const int tau = t + k;
      if (tau < 1 || tau > H) continue;
      const float v = (U[(j + k) * NU + m] - U[(j + k - 1) * NU + m]) * idt;
      const float* du_t = &dU[(j * NU + m) * NZ];
      const float ct = (k == 0 ? idt : -idt);  // d v / d u(t)
      float rows[2] = {w.sq_vel * v, 0.0f}, sc[2] = {w.sq_vel, 0.0f};
      int nr = 1;
      if (w.has_vmax && fabsf(v) > w.v_max) {
        rows[1] = w.sq_lim * (fabsf(v) - w.v_max);
        sc[1] = v < 0.0f ? -w.sq_lim : w.sq_lim;
        nr = 2;
      }
      for (int q = 0; q < nr; ++q) {
        const float r = rows[q], cu = sc[q] * ct;
        if (k == 0) c += 0.5f * r * r;
        for (int a = 0; a < NZ; ++a) g[a] += cu * du_t[a] * r;
        outer(Hs, cu, du_t, cu, du_t);
        if (k == 0) outer(Bk, cu, du_t, -sc[q] * idt, &dU[((j - 1) * NU + m) * NZ]);
      }
    }
    // acceleration rows a(tau) = (u(tau) - 2 u(tau - 1) + u(tau - 2)) / dt^2
    for (int k = 0; k < 3; ++k) {
      const int tau = t + k;
      if (tau < 2 || tau > H) continue;
      const int jt = j + k;  // configuration of tau
      const float a = (U[jt * NU + m] - 2.0f * U[(jt - 1) * NU + m] + U[(jt - 2) * NU + m]) * idt2;
      const float cf[3] = {1.0f, -2.0f, 1.0f};  // coefficient of u(tau - l), l = 0, 1, 2
      const float* du_t = &dU[(j * NU + m) * NZ];
      float rows[2] = {w.sq_acc * a, 0.0f}, sc[2] = {w.sq_acc, 0.0f};
      int nr = 1;
      if (w.has_amax && fabsf(a) > w.a_max) {
        rows[1] = w.sq_lim * (fabsf(a) - w.a_max);
        sc[1] = a < 0.0f ? -w.sq_lim : w.sq_lim;
        nr = 2;
      }
      for (int q = 0; q < nr; ++q) {
        const float r = rows[q], cu = sc[q] * cf[k] * idt2;  // t is tau - k
        if (k == 0) c += 0.5f * r * r;
        for (int aa = 0; aa < NZ; ++aa) g[aa] += cu * du_t[aa] * r;
        outer(Hs, cu, du_t, cu, du_t);
        if (k <= 1 && t >= 1)  // the row also holds t - 1 (coefficient cf[k + 1])
          outer(Bk, cu, du_t, sc[q] * cf[k + 1] * idt2, &dU[((j - 1) * NU + m) * NZ]);
        if (k == 0)  // and t - 2
          outer(Ck, cu, du_t, sc[q] * cf[2] * idt2, &dU[((j - 2) * NU + m) * NZ]);
      }
    }
  }
  if (kind == CR_KIND_TRAJ) {
    // tip path length rows l(tau) = sq_len (p(tau) - p(tau - 1)), tau = t, t + 1
    for (int k = 0; k < 2; ++k) {
      const int tau = t + k;
      if (tau < 1 || tau > H) continue;
      for (int c3 = 0; c3 < 3; ++c3) {
        const float r = w.sq_len * (Pt[(j + k) * 3 + c3] - Pt[(j + k - 1) * 3 + c3]);
        const float cu = k == 0 ? w.sq_len : -w.sq_len;
        const float* dp_t = &dP[(j * 3 + c3) * NZ];
        if (k == 0) c += 0.5f * r * r;
        for (int a = 0; a < NZ; ++a) g[a] += cu * dp_t[a] * r;
        outer(Hs, cu, dp_t, cu, dp_t);
        if (k == 0) outer(Bk, cu, dp_t, -w.sq_len, &dP[((j - 1) * 3 + c3) * NZ]);
      }
    }
    // endpoint rows (eq. 17)
    if (t == 0 || t == H) {
      float ze[NZ];
      b0t_end<NS>(pr, task, rb, t == 0 ? 0 : 1, ze);
      for (int a = 0; a < NZ; ++a) {
        const float r = w.sq_eq * (Z[j * NZ + a] - ze[a]);
        c += 0.5f * r * r;
        g[a] += w.sq_eq * r;
        Hs[a][a] += w.sq_eq * w.sq_eq;
      }
    }
  }
  for (int a = 0; a < NZ; ++a) {
    rec[R::OG + a] = g[a];
    for (int b = 0; b < NZ; ++b) {
      rec[R::OH + b * NZ + a] = Hs[a][b];
      rec[R::OB + b * NZ + a] = Bk[a][b];
      rec[R::OC + b * NZ + a] = Ck[a][b];
    }
  }
  cw[j] += c;
}

// Sum of the waypoint costs of each trajectory; non-finite costs fail it.
__global__ void k_b0t_sum(const TrajProb* __restrict__ row, int S, const float* __restrict__ cw,
                          const float* __restrict__ pw, float* __restrict__ cost, float* __restrict__ pen,
                          int32_t* __restrict__ flags, int mark_failed) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int Tn = row->Tn;
  if (s >= S) return;
  float c = 0.0f, p = 0.0f;
  for (int t = 0; t < Tn; ++t) {
    c += cw[s * Tn + t];
    if (pen) p += pw[s * Tn + t];
  }
  cost[s] = c;
  if (pen) pen[s] = p;
  if (mark_failed && !tfinite(c)) flags[s] |= 1;
}


// One thread per trajectory: damping, block Cholesky of the block-pentadiagonal
// H + lambda D over its records (L blocks overwrite H blocks), forward and
// backward substitution (delta into OY), g.delta.
template <int NS>
__global__ void k_b0t_solve(const TrajProb* __restrict__ row, int S, float* __restrict__ blk,
                            const float* __restrict__ lam, float* __restrict__ gd, int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS;
  using R = B0Rec<NS>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 1)) return;
  const int Tn = row->Tn;
  float* recs = blk + (int64_t)s * Tn * R::SIZE;
  const float l = lam[s];
  bool ok = true;
  auto el = [&](float* rec, int off, int a, int b) -> float& { return rec[off + b * NZ + a]; };  // (row a, col b)
  for (int t = 0; t < Tn; ++t) {
    float* rec = recs + (int64_t)t * R::SIZE;
    float A[NZ][NZ], y[NZ];
    for (int a = 0; a < NZ; ++a) {
      y[a] = -rec[R::OG + a];
      for (int b = 0; b < NZ; ++b) A[a][b] = el(rec, R::OH, a, b);
    }
    for (int a = 0; a < NZ; ++a) A[a][a] += l * (A[a][a] > 1e-12f ? A[a][a] : 1e-12f);
    if (t >= 2) {
      float* r2 = rec - 2 * R::SIZE;  // L_{t-2,t-2} in its OH (lower), y_{t-2} in its OY
      float* r1 = rec - R::SIZE;      // L_{t-1,t-2} in the OB block of record t - 1
      // L_{t,t-2} = H_{t,t-2} L_{t-2,t-2}^-T, row by row
      for (int a = 0; a < NZ; ++a) {
        for (int i = 0; i < NZ; ++i) {
          float v = el(rec, R::OC, a, i);
          for (int k = 0; k < i; ++k) v -= el(rec, R::OC, a, k) * el(r2, R::OH, i, k);
          el(rec, R::OC, a, i) = v / el(r2, R::OH, i, i);
        }
      }
      for (int a = 0; a < NZ; ++a) {
        for (int i = 0; i < NZ; ++i) y[a] -= el(rec, R::OC, a, i) * r2[R::OY + i];
        for (int b = 0; b < NZ; ++b) {
          float v = 0.0f, u = 0.0f;
          for (int i = 0; i < NZ; ++i) {
            v += el(rec, R::OC, a, i) * el(r1, R::OB, b, i);  // L_{t,t-2} L_{t-1,t-2}^T
            u += el(rec, R::OC, a, i) * el(rec, R::OC, b, i);  // L_{t,t-2} L_{t,t-2}^T
          }
          el(rec, R::OB, a, b) -= v;
          A[a][b] -= u;
        }
      }
    }
    if (t >= 1) {
      float* r1 = rec - R::SIZE;  // L_{t-1,t-1} in its OH, y_{t-1} in its OY
      for (int a = 0; a < NZ; ++a) {
        for (int i = 0; i < NZ; ++i) {
          float v = el(rec, R::OB, a, i);
          for (int k = 0; k < i; ++k) v -= el(rec, R::OB, a, k) * el(r1, R::OH, i, k);
          el(rec, R::OB, a, i) = v / el(r1, R::OH, i, i);
        }
      }
      for (int a = 0; a < NZ; ++a) {
        for (int i = 0; i < NZ; ++i) y[a] -= el(rec, R::OB, a, i) * r1[R::OY + i];
        for (int b = 0; b < NZ; ++b) {
          float u = 0.0f;
          for (int i = 0; i < NZ; ++i) u += el(rec, R::OB, a, i) * el(rec, R::OB, b, i);
          A[a][b] -= u;
        }
      }
    }
    // L_tt L_tt^T = A; y_t = L_tt^-1 y
    for (int j = 0; j < NZ; ++j) {
      float d = A[j][j];
      for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
      ok = ok && d > 0.0f;
      const float ljj = sqrtf(d > 0.0f ? d : 1.0f);
      A[j][j] = ljj;
      for (int i = j + 1; i < NZ; ++i) {
        float v = A[i][j];
        for (int k = 0; k < j; ++k) v -= A[i][k] * A[j][k];
        A[i][j] = v / ljj;
      }
    }
    for (int a = 0; a < NZ; ++a) {
      float v = y[a];
      for (int k = 0; k < a; ++k) v -= A[a][k] * y[k];
      y[a] = v / A[a][a];
    }
    for (int a = 0; a < NZ; ++a) {
      rec[R::OY + a] = y[a];
      for (int b = 0; b < NZ; ++b) el(rec, R::OH, a, b) = b <= a ? A[a][b] : 0.0f;
    }
  }
  float gsum = 0.0f;
  for (int t = Tn - 1; t >= 0; --t) {
    float* rec = recs + (int64_t)t * R::SIZE;
    float r[NZ];
    for (int a = 0; a < NZ; ++a) r[a] = rec[R::OY + a];
    if (t + 1 < Tn) {
      const float* q = rec + R::SIZE;  // L_{t+1,t} in OB of t + 1, delta_{t+1} in its OY
      for (int a = 0; a < NZ; ++a)
        for (int b = 0; b < NZ; ++b) r[a] -= q[R::OB + a * NZ + b] * q[R::OY + b];
    }
    if (t + 2 < Tn) {
      const float* q = rec + 2 * R::SIZE;  // L_{t+2,t} in OC of t + 2
      for (int a = 0; a < NZ; ++a)
        for (int b = 0; b < NZ; ++b) r[a] -= q[R::OC + a * NZ + b] * q[R::OY + b];
    }
    for (int a = NZ - 1; a >= 0; --a) {
      float v = r[a];
      for (int k = a + 1; k < NZ; ++k) v -= el(rec, R::OH, k, a) * r[k];
      r[a] = v / el(rec, R::OH, a, a);
    }
    for (int a = 0; a < NZ; ++a) {
      rec[R::OY + a] = r[a];
      gsum += rec[R::OG + a] * r[a];
    }
  }
  gd[s] = gsum;
  flags[s] = (flags[s] & 1) | (ok ? 0 : 4);
}

// Trial point z + alpha delta of every waypoint (keys: alpha = 0, every
// trajectory): its own cost rows in FP32, clearance part apart, lifts and tip.
template <int NS>
__global__ void k_b0t_trial(const TrajProb* __restrict__ row, int S, int kind, RobotT<float> rb, WeightsT<float> w,
                            const double* __restrict__ task, const double* __restrict__ sph, float alpha,
                            const float* __restrict__ Z, const float* __restrict__ blk, float* __restrict__ Zt,
                            float* __restrict__ U, float* __restrict__ Pt, float* __restrict__ cw,
                            float* __restrict__ pw, const int32_t* __restrict__ flags, int keys) {
  constexpr int NZ = 2 * NS, NU = 3 * NS;
  using R = B0Rec<NS>;
  const TrajProb pr = *row;
  const int Tn = pr.Tn, N = S * Tn;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N || (!keys && (flags[j / Tn] & 7))) return;
  const int t = j - (j / Tn) * Tn;
  float z[NZ], u[NU], pt[3];
  for (int k = 0; k < NZ; ++k) {
    z[k] = keys ? Z[j * NZ + k] : Z[j * NZ + k] + alpha * blk[(int64_t)j * R::SIZE + R::OY + k];
    Zt[j * NZ + k] = z[k];
  }
  float Tt[12] = {0};
  if (kind == CR_KIND_PATH) b0t_pose(pr, task, t, Tt);
  float c = 0.0f, cp = 0.0f;
  b0t_rows<NS, float>(rb, w, kind, Tt, sph, pr.sph, pr.sph_ld, pr.M, z, u, pt, [&](float r, bool coll) {
    c += 0.5f * r * r;
    if (coll) cp += 0.5f * r * r;
  });
  for (int m = 0; m < NU; ++m) U[j * NU + m] = u[m];
  for (int c3 = 0; c3 < 3; ++c3) Pt[j * 3 + c3] = pt[c3];
  cw[j] = c;
  pw[j] = cp;
}

// Cost of the coupling rows centred at t, at the trial point (lifts and tips of
// the trial kernel).
template <int NS>
__global__ void k_b0t_tcouple(const TrajProb* __restrict__ row, int S, int kind, RobotT<float> rb, WeightsT<float> w,
                              const double* __restrict__ task, const float* __restrict__ Zt,
                              const float* __restrict__ U, const float* __restrict__ Pt, float* __restrict__ cw,
                              const int32_t* __restrict__ flags, int keys) {
  constexpr int NZ = 2 * NS, NU = 3 * NS;
  const TrajProb pr = *row;
  const int Tn = pr.Tn, H = Tn - 1, N = S * Tn;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N || (!keys && (flags[j / Tn] & 7))) return;
  const int t = j - (j / Tn) * Tn;
  const float idt = 1.0f / w.dt, idt2 = idt * idt;
  float c = 0.0f;
  for (int m = 0; m < NU; ++m) {
    if (t >= 1) {
      const float v = (U[j * NU + m] - U[(j - 1) * NU + m]) * idt;
      const float r = w.sq_vel * v;
      c += 0.5f * r * r;
      if (w.has_vmax && fabsf(v) > w.v_max) {
        const float h = w.sq_lim * (fabsf(v) - w.v_max);
        c += 0.5f * h * h;
      }
    }
    if (t >= 2) {
      const float a = (U[j * NU + m] - 2.0f * U[(j - 1) * NU + m] + U[(j - 2) * NU + m]) * idt2;
      const float r = w.sq_acc * a;
      c += 0.5f * r * r;
      if (w.has_amax && fabsf(a) > w.a_max) {
        const float h = w.sq_lim * (fabsf(a) - w.a_max);
        c += 0.5f * h * h;
      }
    }
  }
  if (kind == CR_KIND_TRAJ) {
    if (t >= 1)
      for (int c3 = 0; c3 < 3; ++c3) {
        const float r = w.sq_len * (Pt[j * 3 + c3] - Pt[(j - 1) * 3 + c3]);
        c += 0.5f * r * r;
      }
    if (t == 0 || t == H) {
      float ze[NZ];
      b0t_end<NS>(pr, task, rb, t == 0 ? 0 : 1, ze);
      for (int a = 0; a < NZ; ++a) {
        const float r = w.sq_eq * (Zt[j * NZ + a] - ze[a]);
        c += 0.5f * r * r;
      }
    }
  }
  cw[j] += c;
}

// Armijo test per trajectory.
__global__ void k_b0t_accept(int S, int trial, float alpha, const float* __restrict__ c0, const float* __restrict__ gd,
                             const float* __restrict__ ct, int32_t* __restrict__ acc, int32_t* __restrict__ flags) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || (flags[s] & 7)) return;
  if (ct[s] <= c0[s] + 1e-4f * alpha * gd[s]) {
    acc[s] = trial;
    flags[s] |= 2;
  }
}

// The trial point of a trajectory accepted at this trial becomes its z.
template <int NS>
__global__ void k_b0t_copy(const TrajProb* __restrict__ row, int S, int trial, const float* __restrict__ Zt,
                           float* __restrict__ Z, const int32_t* __restrict__ acc, const int32_t* __restrict__ flags) {
  constexpr int NZ = 2 * NS;
  const int Tn = row->Tn, N = S * Tn;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int s = j / Tn;
  if ((flags[s] & 3) != 2 || acc[s] != trial) return;
  for (int k = 0; k < NZ; ++k) Z[j * NZ + k] = Zt[j * NZ + k];
}

// Stage-2 start: the kept trajectories, fresh damping.
template <int NS>
__global__ void k_b0t_gather(int Tn, int nf, const float* __restrict__ Z1, const int32_t* __restrict__ sel,
                             float lam0, float* __restrict__ Z2, float* __restrict__ lam, int32_t* __restrict__ flags,
                             int32_t* __restrict__ acc) {
  constexpr int NZ = 2 * NS;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nf * Tn) return;
  const int k = j / Tn, t = j - k * Tn;
  const int s = sel[k];
  for (int m = 0; m < NZ; ++m) Z2[j * NZ + m] = s >= 0 ? Z1[((int64_t)s * Tn + t) * NZ + m] : 0.0f;
  if (t == 0) {
    lam[k] = lam0;
    flags[k] = s >= 0 ? 0 : 1;
    acc[k] = -1;
  }
}


// Host side of the path / trajectory baseline.

struct B0TWs {
  float *Z, *Zt, *Z2, *blk, *U, *dU, *Pt, *dP, *cw, *pw, *lam, *c0, *gd, *ct, *cost, *pen;
  int32_t *flags, *acc, *sel;
  TrajProb* row;
};

static size_t b0t_layout(int ns, int S, int nf, int Tn, char* base, B0TWs* w) {
  const int NZ = 2 * ns, NU = 3 * ns;
  const size_t Sx = S > nf ? S : nf, N = Sx * Tn;
  const size_t rec = 3 * NZ * NZ + 2 * NZ;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t at = off;
    off += (b + 255) & ~(size_t)255;
    return base ? (void*)(base + at) : nullptr;
  };
  B0TWs x{};
  x.Z = (float*)take(4 * N * NZ);
  x.Zt = (float*)take(4 * N * NZ);
  x.Z2 = (float*)take(4 * N * NZ);
  x.blk = (float*)take(4 * N * rec);
  x.U = (float*)take(4 * N * NU);
  x.dU = (float*)take(4 * N * NU * NZ);
  x.Pt = (float*)take(4 * N * 3);
  x.dP = (float*)take(4 * N * 3 * NZ);
  x.cw = (float*)take(4 * N);
  x.pw = (float*)take(4 * N);
  x.lam = (float*)take(4 * Sx);
  x.c0 = (float*)take(4 * Sx);
  x.gd = (float*)take(4 * Sx);
  x.ct = (float*)take(4 * Sx);
  x.cost = (float*)take(4 * Sx);
  x.pen = (float*)take(4 * Sx);
  x.flags = (int32_t*)take(4 * Sx);
  x.acc = (int32_t*)take(4 * Sx);
  x.sel = (int32_t*)take(4 * (size_t)(nf > 0 ? nf : 1));
  x.row = (TrajProb*)take(sizeof(TrajProb));
  if (w) *w = x;
  return off;
}

size_t b0_traj_workspace_bytes(const cr_robot& rb, int S, int H, const cr_opts& o) {
  return b0t_layout(rb.n_seg, S, o.n_final, H + 1, nullptr, nullptr);
}

template <int NS>
static void b0t_stage(int kind, const RobotT<float>& rb, const WeightsT<float>& w, const cr_opts& o,
                      const double* task, const double* sph, int S, int Tn, int iters, const B0TWs& ws, float* Z,
                      hipStream_t st) {
  const dim3 gj((S * Tn + 63) / 64), gs((S + 63) / 64), blk(64);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL((k_b0t_local<NS>), gj, blk, 0, st, ws.row, S, kind, rb, w, task, sph, Z, ws.blk, ws.U,
                       ws.dU, ws.Pt, ws.dP, ws.cw, ws.flags);
    hipLaunchKernelGGL((k_b0t_couple<NS>), gj, blk, 0, st, ws.row, S, kind, rb, w, task, Z, ws.blk, ws.U, ws.dU,
                       ws.Pt, ws.dP, ws.cw, ws.flags);
    hipLaunchKernelGGL(k_b0t_sum, gs, blk, 0, st, ws.row, S, ws.cw, (const float*)nullptr, ws.c0, (float*)nullptr,
                       ws.flags, 1);
    hipLaunchKernelGGL((k_b0t_solve<NS>), gs, blk, 0, st, ws.row, S, ws.blk, ws.lam, ws.gd, ws.flags);
    float alpha = 1.0f;
    for (int tr = 0; tr < o.ls_max; ++tr) {
      hipLaunchKernelGGL((k_b0t_trial<NS>), gj, blk, 0, st, ws.row, S, kind, rb, w, task, sph, alpha, Z, ws.blk,
                         ws.Zt, ws.U, ws.Pt, ws.cw, ws.pw, ws.flags, 0);
      hipLaunchKernelGGL((k_b0t_tcouple<NS>), gj, blk, 0, st, ws.row, S, kind, rb, w, task, ws.Zt, ws.U, ws.Pt,
                         ws.cw, ws.flags, 0);
      hipLaunchKernelGGL(k_b0t_sum, gs, blk, 0, st, ws.row, S, ws.cw, (const float*)nullptr, ws.ct,
                         (float*)nullptr, ws.flags, 0);
      hipLaunchKernelGGL(k_b0t_accept, gs, blk, 0, st, S, tr, alpha, ws.c0, ws.gd, ws.ct, ws.acc, ws.flags);
      hipLaunchKernelGGL((k_b0t_copy<NS>), gj, blk, 0, st, ws.row, S, tr, ws.Zt, Z, ws.acc, ws.flags);
      alpha *= 0.5f;
    }
    hipLaunchKernelGGL(k_b0_lambda, gs, blk, 0, st, S, (float)o.lambda_min, (float)o.lambda_max, ws.lam, ws.acc,
                       ws.flags);
  }
}

// Final cost and clearance part of every trajectory (SelectTop keys, argmin).
template <int NS>
static void b0t_keys(int kind, const RobotT<float>& rb, const WeightsT<float>& w, const double* task,
                     const double* sph, int S, int Tn, const B0TWs& ws, const float* Z, hipStream_t st) {
  const dim3 gj((S * Tn + 63) / 64), gs((S + 63) / 64), blk(64);
  hipLaunchKernelGGL((k_b0t_trial<NS>), gj, blk, 0, st, ws.row, S, kind, rb, w, task, sph, 0.0f, Z, ws.blk, ws.Zt,
                     ws.U, ws.Pt, ws.cw, ws.pw, ws.flags, 1);
  hipLaunchKernelGGL((k_b0t_tcouple<NS>), gj, blk, 0, st, ws.row, S, kind, rb, w, task, ws.Zt, ws.U, ws.Pt, ws.cw,
                     ws.flags, 1);
  hipLaunchKernelGGL(k_b0t_sum, gs, blk, 0, st, ws.row, S, ws.cw, ws.pw, ws.cost, ws.pen, ws.flags, 1);
}

template <int NS>
static cr_status b0t_run(int kind, const cr_robot& rb0, const cr_spheres* sp, int64_t P, int H, const double* task,
                         int S, const double* useed, const cr_weights& w0, const cr_opts& o, double* u_out,
                         double* err_out, int32_t* status_out, const B0TWs& ws, hipStream_t st) {
  const RobotT<float> rb = robot_to<float>(rb0);
  const WeightsT<float> w = weights_to<float>(w0);
  const int Tn = H + 1, nf = o.n_final;
  const int M = sp ? sp->n_sph : 0;
  const double* sph = sp ? (const double*)sp->sph : nullptr;
  cr_status rc = CR_OK;
  for (int64_t q = 0; q < P && rc == CR_OK; ++q) {
    hipLaunchKernelGGL(k_b0t_row, dim3(1), dim3(64), 0, st, kind, P, q, S, Tn, M, sp ? sp->per_problem : 0,
                       sp ? sp->ld : 0, ws.row);
    hipLaunchKernelGGL((k_b0t_init<NS>), dim3((S * Tn + 63) / 64), dim3(64), 0, st, ws.row, useed, rb,
                       (float)o.lambda0, ws.Z, ws.lam, ws.flags, ws.acc);
    b0t_stage<NS>(kind, rb, w, o, task, sph, S, Tn, o.k_init, ws, ws.Z, st);
    b0t_keys<NS>(kind, rb, w, task, sph, S, Tn, ws, ws.Z, st);
    if (nf > 0) {
      rc = launch_select_strided(1, S, 2 * NS * Tn, ws.Z, 1, (int64_t)Tn * 2 * NS, ws.cost, ws.pen, ws.flags, nf,
                                 o.dup_eps, ws.sel, CR_F32, st, nullptr);
      if (rc != CR_OK) break;
      hipLaunchKernelGGL((k_b0t_gather<NS>), dim3((nf * Tn + 63) / 64), dim3(64), 0, st, Tn, nf, ws.Z, ws.sel,
                         (float)o.lambda0, ws.Z2, ws.lam, ws.flags, ws.acc);
      b0t_stage<NS>(kind, rb, w, o, task, sph, nf, Tn, o.k_final, ws, ws.Z2, st);
      b0t_keys<NS>(kind, rb, w, task, sph, nf, Tn, ws, ws.Z2, st);
      rc = launch_traj_assess_f32(kind, rb0, ws.row, task, sph, Tn, nf, ws.sel, ws.Z2, ws.cost, ws.flags, P, u_out,
                                  err_out, status_out, st);
    } else {
      rc = launch_traj_assess_f32(kind, rb0, ws.row, task, sph, Tn, 0, nullptr, ws.Z, ws.cost, ws.flags, P, u_out,
                                  err_out, status_out, st);
    }
    if (rc == CR_OK) rc = check_hip(hipGetLastError(), "trajectory baseline solve");
  }
  return rc;
}

cr_status launch_b0_traj(int kind, const cr_robot& rb, const cr_spheres* sp, int64_t P, int H, const double* task,
                         int S, const double* useed, const cr_weights& w, const cr_opts& o, double* u_out,
                         double* err_out, int32_t* status_out, void* wsmem, hipStream_t st) {
  B0TWs ws;
  b0t_layout(rb.n_seg, S, o.n_final, H + 1, (char*)wsmem, &ws);
#define CR_B0T_CASE(N) \
  case N:              \
    return b0t_run<N>(kind, rb, sp, P, H, task, S, useed, w, o, u_out, err_out, status_out, ws, st);
  switch (rb.n_seg) {
    CR_B0T_CASE(1)
    CR_B0T_CASE(2)
    CR_B0T_CASE(3)
    CR_B0T_CASE(4)
    CR_B0T_CASE(5)
    CR_B0T_CASE(6)
    default:
      return fail(CR_EINVAL, "n_seg out of range");
  }
#undef CR_B0T_CASE
}

}  // namespace crk
