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
                              const double* __restrict__ T, int64_t P, int64_t p, double* __restrict__ u_out,
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
  err_out[p] = pos;
  err_out[P + p] = rot;
  status_out[p] = st == 0 ? CR_SOLVED : st;
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

template <int NS>
static cr_status b0_stage(const RobotT<float>& rb, const WeightsT<float>& w, const cr_opts& o, int S, int iters,
                          const B0Ws& ws, float* z, hipStream_t st) {
  const dim3 grid((S + 63) / 64), blk(64);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL((k_b0_resjac<NS>), grid, blk, 0, st, S, rb, w, ws.Tt, z, ws.r, ws.J, ws.c0, ws.flags);
    hipLaunchKernelGGL((k_b0_normal<NS>), grid, blk, 0, st, S, ws.r, ws.J, ws.Hp, ws.g, ws.flags);
    hipLaunchKernelGGL((k_b0_step<NS>), grid, blk, 0, st, S, ws.Hp, ws.g, ws.lam, ws.dl, ws.gd, ws.flags);
    float alpha = 1.0f;
    for (int tr = 0; tr < o.ls_max; ++tr) {
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
static cr_status b0_run(const cr_robot& rb0, int64_t P, const double* T, int S, const double* useed,
                        const cr_weights& w0, const cr_opts& o, double* u_out, double* err_out, int32_t* status_out,
                        const B0Ws& ws, hipStream_t st) {
  const RobotT<float> rb = robot_to<float>(rb0);
  const WeightsT<float> w = weights_to<float>(w0);
  const RobotT<double> rbd = robot_to<double>(rb0);
  const dim3 grid((S + 63) / 64), blk(64);
  const int nf = o.n_final;
  cr_status rc = CR_OK;
  for (int64_t p = 0; p < P && rc == CR_OK; ++p) {
    hipLaunchKernelGGL(k_b0_target, dim3(1), dim3(64), 0, st, T, P, p, ws.Tt);
    hipLaunchKernelGGL((k_b0_init<NS>), grid, blk, 0, st, S, P * (int64_t)S, p * (int64_t)S, useed, rb,
                       (float)o.lambda0, ws.z, ws.lam, ws.flags);
    hipLaunchKernelGGL(k_b0_fill, grid, blk, 0, st, S, ws.acc, -1);
    rc = b0_stage<NS>(rb, w, o, S, o.k_init, ws, ws.z, st);
    if (rc != CR_OK) break;
    hipLaunchKernelGGL((k_b0_keys<NS>), grid, blk, 0, st, S, rb, w, ws.Tt, ws.z, ws.e, ws.pen, ws.cost, ws.flags);
    if (nf > 0) {
      rc = launch_select(1, S, 2 * NS, ws.z, ws.e, ws.pen, ws.flags, nf, o.dup_eps, ws.sel, CR_F32, st);
      if (rc != CR_OK) break;
      const dim3 g2((nf + 63) / 64);
      hipLaunchKernelGGL((k_b0_gather<NS>), g2, blk, 0, st, S, nf, ws.z, ws.sel, (float)o.lambda0, ws.z2, ws.lam,
                         ws.flags);
      hipLaunchKernelGGL(k_b0_fill, g2, blk, 0, st, nf, ws.acc, -1);
      rc = b0_stage<NS>(rb, w, o, nf, o.k_final, ws, ws.z2, st);
      if (rc != CR_OK) break;
      hipLaunchKernelGGL((k_b0_keys<NS>), g2, blk, 0, st, nf, rb, w, ws.Tt, ws.z2, ws.e, ws.pen, ws.cost, ws.flags);
      hipLaunchKernelGGL((k_b0_finalize<NS>), dim3(1), dim3(64), 0, st, rbd, nf, ws.sel, ws.z2, ws.cost, ws.flags, T,
                         P, p, u_out, err_out, status_out);
    } else {
      hipLaunchKernelGGL((k_b0_finalize<NS>), dim3(1), dim3(64), 0, st, rbd, S, (const int32_t*)nullptr, ws.z,
                         ws.cost, ws.flags, T, P, p, u_out, err_out, status_out);
    }
    rc = check_hip(hipGetLastError(), "baseline solve");
  }
  return rc;
}

cr_status launch_b0_ik(const cr_robot& rb, int64_t P, const double* T, int S, const double* useed,
                       const cr_weights& w, const cr_opts& o, double* u_out, double* err_out, int32_t* status_out,
                       void* wsmem, hipStream_t st) {
  B0Ws ws;
  b0_layout(rb.n_seg, S, o.n_final, (char*)wsmem, &ws);
#define CR_B0_CASE(N) \
  case N:             \
    return b0_run<N>(rb, P, T, S, useed, w, o, u_out, err_out, status_out, ws, st);
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

}  // namespace crk
