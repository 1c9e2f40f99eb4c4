// cr_ik_gen.h -- kernels of the generic per-configuration IK path shared by the
// translation units that instantiate it: stage 1 with clearance rows (spheres,
// self contact) and extensible segments, FP64 stage 2, finalize, and the host
// driver run_ik_gen.  The plain robot's instantiations live in cr_ik.hip, the
// extensible and self-contact ones in cr_ik_ext.hip, cr_ik_self.hip and
// cr_ik_self_ext.hip, so that they compile in parallel.
#pragma once
#include <float.h>

#include "cr_internal.h"

namespace crk {

static inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// Spheres of a solve: sph[c * ld + m] (double), problem p owns columns
// p * M .. p * M + M - 1 when per_problem.
struct SphArgs {
  const double* sph;
  int64_t ld;
  int M, per_problem;
  // convex polytopes (half-space form, see PolyArgs), per problem when per_problem
  const double* pl;
  int64_t pld;
  int NPO, F;
};

// the polytopes of problem p
// Threads of a k_ik_stage2 launch: whole waves per problem, G lanes per candidate.
static inline int64_t stage2_threads(int64_t P, int nf, int G) {
  const int cpw = 64 / G;
  return P * (int64_t)((nf + cpw - 1) / cpw) * 64;
}

__device__ __forceinline__ PolyArgs<double> poly_of(const SphArgs& sa, int64_t p) {
  return PolyArgs<double>{sa.NPO > 0 ? sa.pl + (sa.per_problem ? p * sa.NPO * sa.F : 0) : nullptr, sa.pld, sa.NPO,
                          sa.F};
}

// Stage 1 with clearance rows (eq. 10): one lane per seed as k_ik_stage1, the
// generic per-configuration normal equations; the problem's spheres and polytope
// planes are read by scalar loads (each wave holds seeds of one problem only).
// Also the stage 1 of
// extensible robots (EXT: three coordinates a, b, e per segment), with or
// without spheres (sa.M may be 0).
template <int NS, typename T, bool EXT = false, bool SELF = false, bool POLY = false>
__global__ void __launch_bounds__(256)
    k_ik_stage1_sph(RobotT<T> rb, WeightsT<T> w, LMOpts<T> o, int64_t P, int S, const double* __restrict__ Tt,
                    const double* __restrict__ useed, int iters, T lam0, SphArgs sa, T* __restrict__ z_out,
                    T* __restrict__ e_out, T* __restrict__ pen_out, T* __restrict__ cost_out,
                    int32_t* __restrict__ failed_out, int32_t* __restrict__ trials_out) {
  constexpr int NC = EXT ? 3 : 2, NZ = NC * NS;
  const int64_t B = P * (int64_t)S;
  // ceil(S / 64) waves per problem, so every wave holds seeds of one problem: the
  // problem index and its obstacle pointers are then wave-uniform and the
  // obstacle reads are scalar loads (scalar cache) instead of vector ones
  const int wpp = (S + 63) / 64;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t p = (int64_t)__builtin_amdgcn_readfirstlane((int)(wave / wpp));
  const int s = (int)(wave - (wave / wpp) * wpp) * 64 + (int)(threadIdx.x & 63);
  if (p >= P || s >= S) return;
  const int64_t b = p * S + s;
  const double* sp = sa.M > 0 ? sa.sph + (sa.per_problem ? p * sa.M : 0) : nullptr;
  T tt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) tt[c] = (T)Tt[c * P + p];
  T z[NZ];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const T u0 = (T)useed[(3 * i) * B + b], u1 = (T)useed[(3 * i + 1) * B + b], u2 = (T)useed[(3 * i + 2) * B + b];
    u_to_ab(u0, u1, u2, rb.r[i], &z[NC * i], &z[NC * i + 1]);
    if constexpr (EXT) z[NC * i + 2] = (u0 + u1 + u2) * T(1.0 / 3.0);
  }
  T lam = lam0;
  bool failed = false;
  int trials = 0;
  const PolyArgs<double> po = poly_of(sa, p);
  lm_cfg<NS, T, double, EXT, SELF, 1, POLY>(rb, w, tt, z, lam, iters, o, failed, trials, sp, sa.M, 1, sa.ld, po);
  T e;
  ik_cost<NS, T, EXT>(rb, w, tt, z, &e);
  const T c = cfg_cost<NS, T, double, EXT, SELF, POLY>(rb, w, tt, z, sp, sa.M, 1, sa.ld, po);
  WeightsT<T> wc = w;  // clearance part alone (SelectTop tie-break)
  wc.w_pos = wc.w_rot = wc.sq_lim = wc.sq_curv = T(0);
  const T pen = (sa.M > 0 || SELF || POLY) ? cfg_cost<NS, T, double, EXT, SELF, POLY>(rb, wc, tt, z, sp, sa.M, 1, sa.ld, po)
                                           : T(0);
  if (!tfinite(c) || !tfinite(e)) failed = true;
#pragma unroll
  for (int k = 0; k < NZ; ++k) z_out[k * B + b] = z[k];
  e_out[b] = e;
  pen_out[b] = pen;
  cost_out[b] = c;
  failed_out[b] = failed ? 1 : 0;
  trials_out[b] = trials;
}

// ---------------------------------------------------------------------------
// Stage 2: FP64 refinement of the kept candidates, lambda restarted at lambda0.
// ---------------------------------------------------------------------------

// G lanes per candidate (1, 2 or 4) try the line-search step lengths in
// parallel (lm_cfg); the group leaves together and its first lane writes.
template <int NS, typename T1, bool SPH, bool EXT = false, bool SELF = false, int G = 1, bool POLY = false>
__global__ void __launch_bounds__(256)
    k_ik_stage2(RobotT<double> rb, WeightsT<double> w, LMOpts<double> o, int64_t P, int S, int nf,
                const double* __restrict__ Tt, const T1* __restrict__ z1, const int32_t* __restrict__ sel,
                int iters, double lam0, SphArgs sa, double* __restrict__ z2, double* __restrict__ cost2,
                int32_t* __restrict__ failed2) {
  constexpr int NZ = (EXT ? 3 : 2) * NS, CPW = 64 / G;  // candidates per wave
  const int64_t B2 = P * (int64_t)nf, B1 = P * (int64_t)S;
  // ceil(nf / CPW) waves per problem, so the problem index and its obstacle
  // pointers are wave-uniform (scalar loads), as in k_ik_stage1_sph
  const int wpp = (nf + CPW - 1) / CPW;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t p = (int64_t)__builtin_amdgcn_readfirstlane((int)(wave / wpp));
  const int lanew = (int)(threadIdx.x & 63);
  const int k = (int)(wave - (wave / wpp) * wpp) * CPW + lanew / G;
  const bool lead = lanew % G == 0;
  if (p >= P || k >= nf) return;  // whole groups of G lanes leave together
  const int64_t b = p * nf + k;
  const int s = sel[k * P + p];
  if (s < 0) {
    if (lead) {
#pragma unroll
      for (int m = 0; m < NZ; ++m) z2[m * B2 + b] = 0.0;
      cost2[b] = __builtin_nan("");
      failed2[b] = 1;
    }
    return;
  }
  double tt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) tt[c] = Tt[c * P + p];
  double z[NZ];
#pragma unroll
  for (int m = 0; m < NZ; ++m) z[m] = (double)z1[m * B1 + p * S + s];
  double lam = lam0;
  bool failed = false;
  int trials = 0;
  double c;
  if (SPH || EXT || SELF) {
    const double* sp = sa.M > 0 ? sa.sph + (sa.per_problem ? p * sa.M : 0) : nullptr;
    const PolyArgs<double> po = poly_of(sa, p);
    lm_cfg<NS, double, double, EXT, SELF, G, POLY>(rb, w, tt, z, lam, iters, o, failed, trials, sp, sa.M, 1, sa.ld, po);
    c = cfg_cost<NS, double, double, EXT, SELF, POLY>(rb, w, tt, z, sp, sa.M, 1, sa.ld, po);
  } else {
    lm_ik<NS>(rb, w, tt, z, lam, iters, o, failed, trials);
    c = ik_cost<NS>(rb, w, tt, z, (double*)nullptr);
  }
  if (!tfinite(c)) failed = true;
  if (lead) {
#pragma unroll
    for (int m = 0; m < NZ; ++m) z2[m * B2 + b] = z[m];
    cost2[b] = c;
    failed2[b] = failed ? 1 : 0;
  }
}

// lanes per stage-2 candidate with clearance rows: one wave per SIMD at most
// (256 CUs x 4 SIMDs x 64 lanes), at most four
static inline int stage2_cfg_lanes(int64_t B2) {
  constexpr int64_t kLanes = 256 * 4 * 64;
  return B2 * 4 <= kLanes ? 4 : (B2 * 2 <= kLanes ? 2 : 1);
}


// ---------------------------------------------------------------------------
// Final argmin over candidates and FP64 assessment of the winner.
// Candidates are either the nf stage-2 slots (sel != NULL: seed index sel[k])
// or all S stage-1 seeds (seed index k).
// ---------------------------------------------------------------------------

template <int NS, typename TC, bool EXT = false, bool SELF = false, bool POLY = false>
__global__ void __launch_bounds__(256)
    k_ik_finalize(RobotT<double> rb, int64_t P, int nc, const int32_t* __restrict__ sel,
                  const TC* __restrict__ zc, const TC* __restrict__ costc, const int32_t* __restrict__ failedc,
                  const double* __restrict__ Tt, SphArgs sa, double* __restrict__ u_out, double* __restrict__ err_out,
                  int32_t* __restrict__ status_out) {
  constexpr int NC = EXT ? 3 : 2, NZ = NC * NS;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t Bc = P * (int64_t)nc;
  int best = -1, best_seed = 0;
  double best_cost = 0.0;
  for (int k = 0; k < nc; ++k) {
    const int64_t col = p * nc + k;
    int seed = sel ? sel[k * P + p] : k;
    double c = (double)costc[col];
    if (seed < 0 || failedc[col] || !tfinite(c)) continue;
    if (best < 0 || c < best_cost || (c == best_cost && seed < best_seed)) {
      best = k;
      best_cost = c;
      best_seed = seed;
    }
  }
  if (best < 0) {
    const double nan = __builtin_nan("");
    for (int m = 0; m < 3 * NS; ++m) u_out[m * P + p] = nan;
    err_out[p] = nan;
    err_out[P + p] = nan;
    status_out[p] = CR_NONFINITE;
    return;
  }
  double z[NZ];
#pragma unroll
  for (int m = 0; m < NZ; ++m) z[m] = (double)zc[m * Bc + p * nc + best];
  double tt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) tt[c] = Tt[c * P + p];
  double Rc[9], pc[3];
  fk_tip<NS, double, EXT>(rb, z, Rc, pc);
  double dp[3] = {tt[3] - pc[0], tt[7] - pc[1], tt[11] - pc[2]};
  double pos = sqrt(dot3(dp, dp));
  double Re[9], te[3];
  relative_pose(Rc, pc, tt, Re, te);
  double v[3] = {0.5 * (Re[7] - Re[5]), 0.5 * (Re[2] - Re[6]), 0.5 * (Re[3] - Re[1])};
  double rot = atan2(sqrt(dot3(v, v)), 0.5 * (Re[0] + Re[4] + Re[8] - 1.0));
  double viol = -DBL_MAX, thx = -DBL_MAX;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double u[3];
    ab_to_u(z[NC * i], z[NC * i + 1], rb.r[i], u);
    // extensible: the output carries the extension as the common mode; the tendon
    // bound applies to the bending part, the length to its interval
    const double e = EXT ? z[NC * i + 2] : 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      u_out[(3 * i + j) * P + p] = u[j] + e;
      viol = fmax(viol, fabs(u[j]) - rb.umax[i]);
    }
    if (EXT) viol = fmax(viol, fabs((rb.Ld[i] + e) - rb.Lmidd[i]) - rb.Lhalfd[i]);
    thx = fmax(thx, sqrt(z[NC * i] * z[NC * i] + z[NC * i + 1] * z[NC * i + 1]) - rb.theta_max);
  }
  int32_t st = 0;
  if (viol > 1e-6 || thx > 0.0) st |= CR_LIMIT_VIOLATION;
  if ((sa.M > 0 || SELF || POLY) &&
      penetrates<NS, double, EXT, SELF, POLY>(rb, z, sa.M > 0 ? sa.sph + (sa.per_problem ? p * sa.M : 0) : nullptr, sa.M,
                                              sa.ld, poly_of(sa, p)))
    st |= CR_COLLISION;
  if (!(pos <= 1e-3 && rot <= 3.14159265358979323846 / 180.0)) st |= CR_NOT_CONVERGED;
  if (st == 0) st = CR_SOLVED;
  err_out[p] = pos;
  err_out[P + p] = rot;
  status_out[p] = st;
}

// Algorithm 1 for robots with extensible segments (EXT: three coordinates per
// segment, bending a, b and extension e) or with self contact (SELF: eq. 10 between
// non-adjacent segments); every stage runs the generic per-configuration path
// (clearance rows when spheres are given).
template <int NS, typename T, bool EXT, bool SELF, bool POLY = false>
cr_status run_ik_gen(const cr_robot& rb0, const SphArgs& sa, int64_t P, const double* Tt, int32_t S,
                            const double* useed, const cr_weights& w0, const cr_opts& o, double* u_out,
                            double* err_out, int32_t* status_out, const IkWorkspace& ws, hipStream_t st) {
  RobotT<T> rb = robot_to<T>(rb0);
  WeightsT<T> w = weights_to<T>(w0);
  LMOpts<T> lo{o.ls_max, (T)o.lambda_min, (T)o.lambda_max};
  const int64_t B = P * (int64_t)S;
  const bool timed = timer_on();
  if (timed) timer_begin_call(st);
  hipLaunchKernelGGL((k_ik_stage1_sph<NS, T, EXT, SELF, POLY>), dim3(blocks_for(P * (int64_t)((S + 63) / 64) * 64, 256)),
                     dim3(256), 0, st, rb, w, lo, P, (int)S,
                     Tt, useed, o.k_init, (T)o.lambda0, sa, (T*)ws.z1, (T*)ws.e1, (T*)ws.pen1, (T*)ws.cost1,
                     ws.failed1, ws.trials1);
  cr_status rc = check_hip(hipGetLastError(), "k_ik_stage1_sph");
  if (rc != CR_OK) return rc;
  if (timed) timer_mark(0, st);
  RobotT<double> rbd = robot_to<double>(rb0);
  if (o.n_final > 0) {
    rc = launch_select(P, S, (EXT ? 3 : 2) * NS, ws.z1, ws.e1, ws.pen1, ws.failed1, o.n_final, o.dup_eps, ws.sel,
                       sizeof(T) == 8 ? CR_F64 : CR_F32, st);
    if (rc != CR_OK) return rc;
    if (timed) timer_mark(1, st);
    WeightsT<double> wd = weights_to<double>(w0);
    LMOpts<double> lod{o.ls_max, o.lambda_min, o.lambda_max};
    const int64_t B2 = P * (int64_t)o.n_final;
    const int g2 = stage2_cfg_lanes(B2);
#define CR_S2C(GL)                                                                                                  \
  hipLaunchKernelGGL((k_ik_stage2<NS, T, true, EXT, SELF, GL, POLY>), dim3(blocks_for(stage2_threads(P, o.n_final, GL), 256)), \
                     dim3(256), 0, st, rbd, \
                     wd, lod, P, (int)S, (int)o.n_final, Tt, (const T*)ws.z1, ws.sel, o.k_final, o.lambda0, sa, ws.z2, \
                     ws.cost2, ws.failed2)
    if (g2 == 4) CR_S2C(4);
    else if (g2 == 2) CR_S2C(2);
    else CR_S2C(1);
#undef CR_S2C
    rc = check_hip(hipGetLastError(), "k_ik_stage2");
    if (rc != CR_OK) return rc;
    if (timed) timer_mark(2, st);
    hipLaunchKernelGGL((k_ik_finalize<NS, double, EXT, SELF, POLY>), dim3(blocks_for(P, 256)), dim3(256), 0, st, rbd, P,
                       (int)o.n_final, ws.sel, ws.z2, ws.cost2, ws.failed2, Tt, sa, u_out, err_out, status_out);
  } else {
    if (timed) {
      timer_mark(1, st);
      timer_mark(2, st);
    }
    hipLaunchKernelGGL((k_ik_finalize<NS, T, EXT, SELF, POLY>), dim3(blocks_for(P, 256)), dim3(256), 0, st, rbd, P, (int)S,
                       (const int32_t*)nullptr, (const T*)ws.z1, (const T*)ws.cost1, ws.failed1, Tt, sa, u_out,
                       err_out, status_out);
  }
  rc = check_hip(hipGetLastError(), "k_ik_finalize");
  if (timed) {
    timer_mark(3, st);
    timer_end_call();
  }
  return rc;
}

#define CR_IK_GEN_INST(EXT, SELF, NS)                                                                              \
  template cr_status run_ik_gen<NS, float, EXT, SELF>(const cr_robot&, const SphArgs&, int64_t, const double*,    \
                                                       int32_t, const double*, const cr_weights&, const cr_opts&, \
                                                       double*, double*, int32_t*, const IkWorkspace&, hipStream_t); \
  template cr_status run_ik_gen<NS, double, EXT, SELF>(const cr_robot&, const SphArgs&, int64_t, const double*,   \
                                                        int32_t, const double*, const cr_weights&, const cr_opts&, \
                                                        double*, double*, int32_t*, const IkWorkspace&, hipStream_t);
#define CR_IK_GEN_INST_POLY(NS)                                                                                    \
  template cr_status run_ik_gen<NS, float, false, false, true>(const cr_robot&, const SphArgs&, int64_t,           \
                                                               const double*, int32_t, const double*,              \
                                                               const cr_weights&, const cr_opts&, double*, double*, \
                                                               int32_t*, const IkWorkspace&, hipStream_t);          \
  template cr_status run_ik_gen<NS, double, false, false, true>(const cr_robot&, const SphArgs&, int64_t,          \
                                                                const double*, int32_t, const double*,             \
                                                                const cr_weights&, const cr_opts&, double*,         \
                                                                double*, int32_t*, const IkWorkspace&, hipStream_t);
#define CR_IK_GEN_EXTERN_POLY(NS)                                                                                  \
  extern template cr_status run_ik_gen<NS, float, false, false, true>(const cr_robot&, const SphArgs&, int64_t,    \
                                                                      const double*, int32_t, const double*,       \
                                                                      const cr_weights&, const cr_opts&, double*,   \
                                                                      double*, int32_t*, const IkWorkspace&,        \
                                                                      hipStream_t);                                 \
  extern template cr_status run_ik_gen<NS, double, false, false, true>(const cr_robot&, const SphArgs&, int64_t,   \
                                                                       const double*, int32_t, const double*,      \
                                                                       const cr_weights&, const cr_opts&, double*,  \
                                                                       double*, int32_t*, const IkWorkspace&,       \
                                                                       hipStream_t);
#define CR_IK_GEN_EXTERN(EXT, SELF, NS)                                                                            \
  extern template cr_status run_ik_gen<NS, float, EXT, SELF>(const cr_robot&, const SphArgs&, int64_t,            \
                                                              const double*, int32_t, const double*,              \
                                                              const cr_weights&, const cr_opts&, double*, double*, \
                                                              int32_t*, const IkWorkspace&, hipStream_t);          \
  extern template cr_status run_ik_gen<NS, double, EXT, SELF>(const cr_robot&, const SphArgs&, int64_t,           \
                                                               const double*, int32_t, const double*,             \
                                                               const cr_weights&, const cr_opts&, double*, double*, \
                                                               int32_t*, const IkWorkspace&, hipStream_t);

}  // namespace crk
