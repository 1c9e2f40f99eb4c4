// cr_tally.hip -- algorithmic operation counts of the IK stage-1 kernel.
//
// The stage-1 arithmetic in cr_device.h is templated on its scalar type.  Here
// it is replayed on the host with CountT, an FP32 value that counts every
// floating operation it performs, over a caller-given sample of seeds.  The counts
// are therefore those of the kernel's own formulas, taking the kernel's branches
// and line-search trials in the kernel's precision (up to the rounding of fused
// multiply-adds and of the host's math library), not an estimate.  Counting rules:
// add, sub, mul = 1 each (a fused multiply-add counts as its mul and its add,
// i.e. 2); div, sqrt and the transcendental calls (sin and cos of sincos count
// 2, atan2 1) are tallied separately and count 1 flop each in the total.
#include <math.h>

#include "cr_internal.h"

namespace crk {

struct OpCount {
  double addmul, div, sqrt, trans;
};
static thread_local OpCount g_ops;

struct CountT {
  float v;
  CountT() : v(0.0f) {}
  CountT(double x) : v((float)x) {}
  explicit operator double() const { return (double)v; }
};
inline CountT operator+(CountT a, CountT b) { g_ops.addmul += 1; return CountT(a.v + b.v); }
inline CountT operator-(CountT a, CountT b) { g_ops.addmul += 1; return CountT(a.v - b.v); }
inline CountT operator*(CountT a, CountT b) { g_ops.addmul += 1; return CountT(a.v * b.v); }
inline CountT operator/(CountT a, CountT b) { g_ops.div += 1; return CountT(a.v / b.v); }
inline CountT operator-(CountT a) { return CountT(-a.v); }
inline CountT& operator+=(CountT& a, CountT b) { a = a + b; return a; }
inline CountT& operator-=(CountT& a, CountT b) { a = a - b; return a; }
inline CountT& operator*=(CountT& a, CountT b) { a = a * b; return a; }
inline bool operator<(CountT a, CountT b) { return a.v < b.v; }
inline bool operator>(CountT a, CountT b) { return a.v > b.v; }
inline bool operator<=(CountT a, CountT b) { return a.v <= b.v; }
inline bool operator>=(CountT a, CountT b) { return a.v >= b.v; }
inline bool operator==(CountT a, CountT b) { return a.v == b.v; }
inline bool operator!=(CountT a, CountT b) { return a.v != b.v; }
inline CountT fabs(CountT a) { return CountT(::fabsf(a.v)); }

template <>
CR_HD CountT tsqrt<CountT>(CountT x) {
  g_ops.sqrt += 1;
  return CountT(::sqrtf(x.v));
}
template <>
CR_HD CountT tatan2<CountT>(CountT y, CountT x) {
  g_ops.trans += 1;
  return CountT(::atan2f(y.v, x.v));
}
template <>
CR_HD void tsincos<CountT>(CountT x, CountT* s, CountT* c) {
  g_ops.trans += 2;
  *s = CountT(::sinf(x.v));
  *c = CountT(::cosf(x.v));
}
template <>
CR_HD bool tfinite<CountT>(CountT x) {
  return isfinite(x.v);
}
// the FP32 kernel's series lengths and switch points
template <>
struct Prec<CountT> {
  static constexpr int NT = Prec<float>::NT;
  static constexpr double s_switch = Prec<float>::s_switch;
  static constexpr int NG = Prec<float>::NG;
  static constexpr double g_switch = Prec<float>::g_switch;
};

static double total(const OpCount& c) { return c.addmul + c.div + c.sqrt + c.trans; }

template <int NS>
static void tally_ik(const cr_robot& rb0, const cr_weights& w0, const cr_opts& o, int64_t n, const double* T,
                     const double* u, double* out) {
  RobotT<double> rd = robot_to<double>(rb0);
  WeightsT<double> wd = weights_to<double>(w0);
  RobotT<CountT> rb;
  rb.n = rd.n;
  rb.K = rd.K;
  for (int i = 0; i < CR_MAX_SEG; ++i) {
    rb.L[i] = rd.L[i];
    rb.r[i] = rd.r[i];
    rb.umax[i] = rd.umax[i];
  }
  rb.theta_max = rd.theta_max;
  for (int i = 0; i < CR_MAX_SEG; ++i) {
    rb.Ld[i] = rd.Ld[i];
    rb.rd[i] = rd.rd[i];
    rb.umaxd[i] = rd.umaxd[i];
  }
  rb.theta_maxd = rd.theta_maxd;
  WeightsT<CountT> w;
  w.w_pos = wd.w_pos; w.w_rot = wd.w_rot; w.sq_lim = wd.sq_lim; w.sq_curv = wd.sq_curv;
  w.sq_coll = wd.sq_coll; w.margin = wd.margin; w.sq_eq = wd.sq_eq; w.sq_len = wd.sq_len;
  w.sq_vel = wd.sq_vel; w.sq_acc = wd.sq_acc; w.v_max = wd.v_max; w.a_max = wd.a_max; w.dt = wd.dt;
  w.has_vmax = wd.has_vmax; w.has_amax = wd.has_amax; w.margind = wd.margind;
  LMOpts<CountT> lo{o.ls_max, CountT((double)(float)o.lambda_min), CountT((double)(float)o.lambda_max)};
  OpCount sum{0, 0, 0, 0};
  double trials_sum = 0.0, one_neq = 0.0, one_cost = 0.0;
  for (int64_t s = 0; s < n; ++s) {
    CountT tt[12], z[2 * NS];
    for (int c = 0; c < 12; ++c) tt[c] = CountT(T[s * 12 + c]);
    g_ops = OpCount{0, 0, 0, 0};
    for (int i = 0; i < NS; ++i)
      u_to_ab(CountT(u[s * 3 * NS + 3 * i]), CountT(u[s * 3 * NS + 3 * i + 1]), CountT(u[s * 3 * NS + 3 * i + 2]),
              rb.r[i], &z[2 * i], &z[2 * i + 1]);
    if (s == 0) {
      OpCount save = g_ops;
      CountT Hp[2 * NS * (2 * NS + 1) / 2], g[2 * NS];
      g_ops = OpCount{0, 0, 0, 0};
      ik_normal_eq<NS>(rb, w, tt, z, Hp, g);
      one_neq = total(g_ops);
      g_ops = OpCount{0, 0, 0, 0};
      ik_cost<NS>(rb, w, tt, z, (CountT*)nullptr);
      one_cost = total(g_ops);
      g_ops = save;
    }
    CountT lam((double)(float)o.lambda0);
    bool failed = false;
    int trials = 0;
    lm_ik<NS>(rb, w, tt, z, lam, o.k_init, lo, failed, trials);
    CountT e;
    ik_cost<NS>(rb, w, tt, z, &e);
    sum.addmul += g_ops.addmul;
    sum.div += g_ops.div;
    sum.sqrt += g_ops.sqrt;
    sum.trans += g_ops.trans;
    trials_sum += trials;
  }
  const double inv = n > 0 ? 1.0 / (double)n : 0.0;
  out[0] = total(sum) * inv;
  out[1] = sum.addmul * inv;
  out[2] = sum.div * inv;
  out[3] = sum.sqrt * inv;
  out[4] = sum.trans * inv;
  out[5] = trials_sum * inv;
  out[6] = one_neq;
  out[7] = one_cost;
}

cr_status tally_ik_dispatch(const cr_robot& rb, const cr_weights& w, const cr_opts& o, int64_t n, const double* T,
                            const double* u, double* out) {
  switch (rb.n_seg) {
    case 1: tally_ik<1>(rb, w, o, n, T, u, out); break;
    case 2: tally_ik<2>(rb, w, o, n, T, u, out); break;
    case 3: tally_ik<3>(rb, w, o, n, T, u, out); break;
    case 4: tally_ik<4>(rb, w, o, n, T, u, out); break;
    case 5: tally_ik<5>(rb, w, o, n, T, u, out); break;
    case 6: tally_ik<6>(rb, w, o, n, T, u, out); break;
    default: return fail(CR_EINVAL, "n_seg out of range");
  }
  return CR_OK;
}

}  // namespace crk
