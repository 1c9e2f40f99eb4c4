// cr_ik.hip -- two-stage inverse kinematics (Algorithm 1) on gfx950.
//
//   k_ik_stage1   one lane per seed: k_init LM iterations in the stage-1 type
//                 (FP32 bulk or FP64), then the seed's unweighted pose error
//                 (SelectTop key), collision penalty and final cost
//   k_select      one workgroup per problem: LDS bitonic sort + greedy
//                 near-duplicate pass (SelectTop)
//   k_ik_stage2   one lane per kept candidate: k_final LM iterations in FP64
//   k_ik_finalize one lane per problem: argmin of the final cost (ties to the
//                 lower seed index), FP64 assessment and zero-sum output
//
// All per-seed state stays in VGPRs for the whole iteration loop; HBM sees the
// seeds once and the per-seed summaries once.
#include "cr_ik_gen.h"

namespace crk {

CR_IK_GEN_EXTERN_POLY(1)
CR_IK_GEN_EXTERN_POLY(2)
CR_IK_GEN_EXTERN_POLY(3)
CR_IK_GEN_EXTERN_POLY(4)
CR_IK_GEN_EXTERN_POLY(5)
CR_IK_GEN_EXTERN_POLY(6)
CR_IK_GEN_EXTERN(true, false, 1)
CR_IK_GEN_EXTERN(true, false, 2)
CR_IK_GEN_EXTERN(true, false, 3)
CR_IK_GEN_EXTERN(true, false, 4)
CR_IK_GEN_EXTERN(true, false, 5)
CR_IK_GEN_EXTERN(true, false, 6)
CR_IK_GEN_EXTERN(false, true, 3)
CR_IK_GEN_EXTERN(true, true, 3)
CR_IK_GEN_EXTERN(false, true, 4)
CR_IK_GEN_EXTERN(true, true, 4)
CR_IK_GEN_EXTERN(false, true, 5)
CR_IK_GEN_EXTERN(true, true, 5)
CR_IK_GEN_EXTERN(false, true, 6)
CR_IK_GEN_EXTERN(true, true, 6)

// OCC: the minimum waves per SIMD the register allocation must allow (1 = the
// compiler's own choice); the autotuner picks among the compiled targets.
template <int NS, typename T, int OCC = 1>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC)))
    k_ik_stage1(RobotT<T> rb, WeightsT<T> w, LMOpts<T> o, int64_t P, int S, const double* __restrict__ Tt,
                const double* __restrict__ useed, int iters, T lam0, T* __restrict__ z_out, T* __restrict__ e_out,
                T* __restrict__ pen_out, T* __restrict__ cost_out, int32_t* __restrict__ failed_out,
                int32_t* __restrict__ trials_out) {
  constexpr int NZ = 2 * NS;
  const int64_t B = P * (int64_t)S;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int64_t p = b / S;
  T tt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) tt[c] = (T)Tt[c * P + p];
  T z[NZ];
#pragma unroll
  for (int i = 0; i < NS; ++i)
    u_to_ab((T)useed[(3 * i) * B + b], (T)useed[(3 * i + 1) * B + b], (T)useed[(3 * i + 2) * B + b], rb.r[i],
            &z[2 * i], &z[2 * i + 1]);
  T lam = lam0;
  bool failed = false;
  int trials = 0;
  lm_ik<NS>(rb, w, tt, z, lam, iters, o, failed, trials);
  T e;
  T c = ik_cost<NS>(rb, w, tt, z, &e);
  if (!tfinite(c) || !tfinite(e)) failed = true;
#pragma unroll
  for (int k = 0; k < NZ; ++k) z_out[k * B + b] = z[k];
  e_out[b] = e;
  pen_out[b] = T(0);
  cost_out[b] = c;
  failed_out[b] = failed ? 1 : 0;
  trials_out[b] = trials;
}

// ---------------------------------------------------------------------------
// SelectTop.  Keys (flag, e, index) are sorted ascending in LDS by a bitonic
// network (flag 0 = valid, 1 = failed, 2 = padding); all keys are distinct, so
// the order equals a stable sort by (flag, e).  The first wave then walks the
// order: each candidate is compared with every kept one at once, one lane per
// (kept candidate, coordinate) pair, and the walk's decisions are uniform across
// the wave.  The candidates' coordinates are staged in LDS when they fit.
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ bool key_less(T ea, int fa, T eb, int fb) {
  // fa/fb pack (flag << 16) | index
  int ga = fa >> 16, gb = fb >> 16;
  if (ga != gb) return ga < gb;
  if (ga == 0 && ea != eb) return ea < eb;
  return (fa & 0xffff) < (fb & 0xffff);
}

// LDS of k_select for up to Spad candidates, with room to stage the penalties
// (stage_pen) and stage_nz coordinates per candidate (0: coordinates are read
// from z).
static inline size_t select_lds(int Spad, int stage_pen, int stage_nz, size_t tb) {
  size_t b = (size_t)Spad * ((stage_pen ? 2 : 1) * tb + 4) + (size_t)Spad;
  b = (b + 7) & ~(size_t)7;
  b += 64 * 4;
  return b + (size_t)Spad * stage_nz * tb;
}

// Candidate c of problem p, coordinate m is z[m * zs_m + (p * S + c) * zc] and
// its keys sit at p * S + c; with rows != NULL problem p has its own candidate
// count, key base and z layout (ragged batches, trajectories).
// SelectTop of problem p by the calling workgroup (any multiple of 64 lanes; its
// first wave takes the decisions); row: that problem's own candidate layout, or
// NULL for the uniform one.  smem: select_lds() bytes.
template <typename T>
__device__ void select_top_one(int64_t P, int64_t p, int S0, int Spad0, int nz0, int stage_pen, int stage_nz,
                               const T* __restrict__ z, int64_t zs_m, int64_t zs_c, const T* __restrict__ e,
                               const T* __restrict__ pen, const int32_t* __restrict__ failed, int n_final, T dup_eps,
                               const SelRow* row, int32_t* __restrict__ idx_out, unsigned char* smem) {
  T* se = reinterpret_cast<T*>(smem);
  T* spen = se + Spad0;  // penalties for the duplicate rule, when staged
  int* sf = reinterpret_cast<int*>(stage_pen ? spen + Spad0 : spen);
  unsigned char* skipped = reinterpret_cast<unsigned char*>(sf + Spad0);
  int* kept = reinterpret_cast<int*>(
      smem + ((((size_t)Spad0 * ((stage_pen ? 2 : 1) * sizeof(T) + 4) + Spad0) + 7) & ~(size_t)7));
  T* sz = reinterpret_cast<T*>(kept + 64);
  int S = S0, nz = nz0, Spad = Spad0;
  int64_t kb = p * S0, zb = p * S0 * zs_c, zc = zs_c;
  if (row) {
    const SelRow r = *row;
    S = r.S;
    nz = r.nz;
    kb = r.kbase;
    zb = r.zbase;
    zc = r.zsc;
    Spad = 1;
    while (Spad < S) Spad <<= 1;
  }
  const bool staged = nz <= stage_nz;
  for (int i = threadIdx.x; i < Spad; i += blockDim.x) {
    if (i < S) {
      T ev = e[kb + i];
      int fl = (failed && failed[kb + i] == 1) || !tfinite(ev) ? 1 : 0;
      se[i] = ev;
      if (stage_pen) spen[i] = pen[kb + i];
      sf[i] = (fl << 16) | i;
    } else {
      se[i] = T(0);
      sf[i] = (2 << 16) | i;
    }
    skipped[i] = 0;
  }
  if (staged) {
    // consecutive threads read consecutive candidates of one coordinate
    for (int i = threadIdx.x; i < S * nz; i += blockDim.x) {
      const int m = i / S, c = i - m * S;
      sz[c * nz + m] = z[zb + m * zs_m + c * zc];
    }
  }
  __syncthreads();
  for (int k = 2; k <= Spad; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < Spad; i += blockDim.x) {
        int l = i ^ j;
        if (l > i) {
          bool up = (i & k) == 0;
          T ei = se[i], el = se[l];
          int fi = sf[i], fl = sf[l];
          bool swap = up ? key_less(el, fl, ei, fi) : key_less(ei, fi, el, fl);
          if (swap) {
            se[i] = el;
            se[l] = ei;
            sf[i] = fl;
            sf[l] = fi;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x >= 64) return;
  // One wave from here on.  Every lane takes the same decisions and writes the same
  // values to the kept list and the skip flags, so the wave's in-order LDS accesses
  // keep them consistent without a barrier.
  const int lane = (int)threadIdx.x;
  auto coord = [&](int c, int m) -> T { return staged ? sz[c * nz + m] : z[zb + m * zs_m + c * zc]; };
  auto penalty = [&](int c) -> T { return stage_pen ? spen[c] : pen[kb + c]; };
  int nk = 0;
  if (nz <= 16) {
    // Short candidates: 64 candidates at a time, one per lane, each tested against
    // the kept set; the decisions that change the kept set (a new distinct
    // candidate, a duplicate with a lower penalty) are taken in order, and the
    // lanes after each one are tested again, so every decision sees the kept set
    // that the candidate-by-candidate rule would.
    // A NaN difference never counts as far, as in a running maximum that skips NaN.
    auto first_dup = [&](int c) -> int {
      for (int k = 0; k < nk; ++k) {
        const int ck = kept[k];
        bool far = false;
        for (int m = 0; m < nz; ++m) far = far || (fabs(coord(c, m) - coord(ck, m)) > dup_eps);
        if (!far) return k;
      }
      return -1;
    };
    bool last = false;
    for (int base = 0; base < S && nk < n_final && !last; base += 64) {
      const int q = base + lane;
      const int f = q < S ? sf[q] : (2 << 16);
      const bool valid = (f >> 16) == 0;  // the valid candidates are a prefix of the order
      const int c = f & 0xffff;
      last = __ballot(!valid) != 0ull;
      int dup = valid ? first_dup(c) : -1;
      int i = 0;  // first lane not decided yet
      while (i < 64 && nk < n_final) {
        const bool open = valid && lane >= i;
        const bool ev = open && (dup < 0 || penalty(c) < penalty(kept[dup]));
        const unsigned long long em = __ballot(ev);
        if (em == 0ull) {
          if (open) skipped[c] = 1;
          break;
        }
        const int j = __builtin_ctzll(em);
        if (open && lane < j) skipped[c] = 1;
        const int cj = __shfl(c, j, 64), dj = __shfl(dup, j, 64);
        if (dj < 0) {
          kept[nk] = cj;
          ++nk;
        } else {
          skipped[kept[dj]] = 1;
          kept[dj] = cj;
        }
        i = j + 1;
        if (valid && lane >= i) dup = first_dup(c);
      }
    }
  } else {
    // Long candidates (trajectories): one candidate at a time, all lanes comparing
    // it with the kept ones, one lane per (kept candidate, coordinate) pair.
    for (int q = 0; q < S && nk < n_final; ++q) {
      const int f = sf[q];
      if ((f >> 16) != 0) break;
      const int c = f & 0xffff;
      // bit k: some coordinate differs from kept candidate k by more than dup_eps
      // (a NaN difference never counts, as in a running maximum that skips NaN)
      unsigned long long kfar = 0ull;
      const int np = nk * nz;
      for (int base = 0; base < np; base += 64) {
        const int pi = base + lane;
        bool far = false;
        if (pi < np) {
          const int k = pi / nz, m = pi - k * nz;
          far = fabs(coord(c, m) - coord(kept[k], m)) > dup_eps;
        }
        const unsigned long long fm = __ballot(far);
        if (fm != 0ull) {
          const int k0 = base / nz;
          const int k1 = (base + 63) / nz < nk - 1 ? (base + 63) / nz : nk - 1;
          for (int k = k0; k <= k1; ++k) {
            const int lo = k * nz - base > 0 ? k * nz - base : 0;
            const int hi = (k + 1) * nz - base < 64 ? (k + 1) * nz - base : 64;
            const unsigned long long win = (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull)) & ~((1ull << lo) - 1ull);
            if (fm & win) kfar |= 1ull << k;
          }
        }
      }
      const unsigned long long near = ~kfar & (nk >= 64 ? ~0ull : ((1ull << nk) - 1ull));
      if (near == 0ull) {
        kept[nk] = c;
        ++nk;
      } else {
        const int dup = __builtin_ctzll(near);  // the first kept candidate it duplicates
        const int kd = kept[dup];
        if ((stage_pen ? spen[c] : pen[kb + c]) < (stage_pen ? spen[kd] : pen[kb + kd])) {
          skipped[kd] = 1;
          kept[dup] = c;
        } else {
          skipped[c] = 1;
        }
      }
    }
  }
  // Not enough distinct candidates: the skipped ones fill up the list in order.
  for (int base = 0; base < S && nk < n_final; base += 64) {
    const int q = base + lane;
    const int f = q < S ? sf[q] : (2 << 16);
    const bool valid = (f >> 16) == 0;
    const int c = f & 0xffff;
    const bool take = valid && skipped[c];
    const unsigned long long tm = __ballot(take);
    const int rank =
        (int)__builtin_amdgcn_mbcnt_hi((unsigned)(tm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)tm, 0u));
    if (take && nk + rank < n_final) kept[nk + rank] = c;
    nk = nk + __popcll(tm) < n_final ? nk + __popcll(tm) : n_final;
    if (__ballot(!valid) != 0ull) break;
  }
  if (lane < n_final) idx_out[(int64_t)lane * P + p] = lane < nk ? kept[lane] : -1;
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_select(int64_t P, int S0, int Spad0, int nz0, int stage_pen, int stage_nz, const T* __restrict__ z, int64_t zs_m,
             int64_t zs_c, const T* __restrict__ e, const T* __restrict__ pen, const int32_t* __restrict__ failed,
             int n_final, T dup_eps, const SelRow* __restrict__ rows, int32_t* __restrict__ idx_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t p = blockIdx.x;
  select_top_one<T>(P, p, S0, Spad0, nz0, stage_pen, stage_nz, z, zs_m, zs_c, e, pen, failed, n_final, dup_eps,
                    rows ? rows + p : nullptr, idx_out, smem);
}

// Stage 2 for robots without clearance rows, G lanes per kept candidate (G = 1, 2
// or 4).  One lane per candidate leaves SIMDs idle when the candidates are few
// (32,768 candidates are 512 waves for 1024 SIMDs), and a wave with half its lanes
// active issues no faster than a full one.  Here the G lanes of a group carry the
// same candidate: each forms the same normal equations and step (identical inputs
// and instructions, so identical values), and the line search evaluates G step
// lengths at once, lane q taking alpha = 2^-(G r + q) in round r; the accepted
// step is the first that passes in the sequential order, found with a ballot over
// the group.  Decisions and iterates are those of lm_ik.
// lanes of one wave per SIMD over the whole chip: 256 CUs x 4 SIMDs x 64 lanes
constexpr int64_t kStage2Lanes = 256 * 4 * 64;

template <int NS, typename T1, int G>
__global__ void __launch_bounds__(256)
    k_ik_stage2_grp(RobotT<double> rb, WeightsT<double> w, LMOpts<double> o, int64_t P, int S, int nf,
                    const double* __restrict__ Tt, const T1* __restrict__ z1, const int32_t* __restrict__ sel,
                    int iters, double lam0, double* __restrict__ z2, double* __restrict__ cost2,
                    int32_t* __restrict__ failed2) {
  static_assert(G == 1 || G == 2 || G == 4, "group of 1, 2 or 4 lanes");
  constexpr int NZ = 2 * NS, NP = NZ * (NZ + 1) / 2;
  const int64_t B2 = P * (int64_t)nf, B1 = P * (int64_t)S;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = t / G;
  const int q = (int)(t % G);
  if (b >= B2) return;  // the whole group leaves together
  const int64_t p = b / nf;
  const int k = (int)(b % nf);
  const int s = sel[k * P + p];
  if (s < 0) {
    if (q == 0) {
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
  const int lane = threadIdx.x & 63, base = lane & ~(G - 1);
  const int rounds = (o.ls_max + G - 1) / G;
  for (int it = 0; it < iters; ++it) {
    double Hp[NP], g[NZ], dl[NZ];
    const double c0 = ik_normal_eq<NS>(rb, w, tt, z, Hp, g);
    if (!tfinite(c0)) {
      failed = true;
      break;
    }
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      const double hj = Hp[tri(j, j)];
      Hp[tri(j, j)] = hj + lam * (hj > 1e-12 ? hj : 1e-12);
      dl[j] = -g[j];
    }
    if (!chol_solve<NZ>(Hp, dl)) {
      if (!(lam < o.lam_max)) break;
      lam = lam * 10.0 < o.lam_max ? lam * 10.0 : o.lam_max;
      continue;
    }
    double gd = 0.0;
#pragma unroll
    for (int j = 0; j < NZ; ++j) gd += g[j] * dl[j];
    int acc = -1;
    for (int r = 0; r < rounds && acc < 0; ++r) {
      const int tr = G * r + q;
      bool ok = false;
      if (tr < o.ls_max) {
        const double alpha = ldexp(1.0, -tr);
        double zt[NZ];
#pragma unroll
        for (int j = 0; j < NZ; ++j) zt[j] = z[j] + alpha * dl[j];
        const double c = ik_cost<NS>(rb, w, tt, zt, (double*)nullptr);
        ok = c <= c0 + 1e-4 * alpha * gd;
      }
      const unsigned grp = (unsigned)((__ballot(ok) >> base) & ((1ull << G) - 1));
      if (grp) acc = G * r + __builtin_ctz(grp);
    }
    if (acc >= 0) {
      const double alpha = ldexp(1.0, -acc);
#pragma unroll
      for (int j = 0; j < NZ; ++j) z[j] = z[j] + alpha * dl[j];
      if (acc == 0) lam = lam / 10.0 > o.lam_min ? lam / 10.0 : o.lam_min;
    } else {
      if (!(lam < o.lam_max)) break;
      lam = lam * 10.0 < o.lam_max ? lam * 10.0 : o.lam_max;
    }
  }
  const double c = ik_cost<NS>(rb, w, tt, z, (double*)nullptr);
  if (!tfinite(c)) failed = true;
  if (q == 0) {
#pragma unroll
    for (int m = 0; m < NZ; ++m) z2[m * B2 + b] = z[m];
    cost2[b] = c;
    failed2[b] = failed ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Ragged launches (uneven batches): every problem has its own seed count,
// sphere set and array offsets (struct IkProb); same per-seed iteration.
// ---------------------------------------------------------------------------

// Stage 1 of seed s of problem pr (the seed at b in the launch's stage-1 arrays).
template <int NS, typename T>
__device__ __forceinline__ void ik_rag_seed(const RobotT<T>& rb, const WeightsT<T>& w, const LMOpts<T>& o,
                                            const IkProb& pr, int64_t b, int64_t s, int64_t B,
                                            const double* __restrict__ task, const double* __restrict__ useed,
                                            const double* __restrict__ sph, int iters, T lam0, T* __restrict__ z_out,
                                            T* __restrict__ e_out, T* __restrict__ pen_out, T* __restrict__ cost_out,
                                            int32_t* __restrict__ failed_out) {
  constexpr int NZ = 2 * NS;
  T tt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) tt[c] = (T)task[pr.task + c * pr.task_ld];
  T z[NZ];
  const double* u = useed + pr.seed + s;
#pragma unroll
  for (int i = 0; i < NS; ++i)
    u_to_ab((T)u[(3 * i) * pr.seed_ld], (T)u[(3 * i + 1) * pr.seed_ld], (T)u[(3 * i + 2) * pr.seed_ld], rb.r[i],
            &z[2 * i], &z[2 * i + 1]);
  T lam = lam0;
  bool failed = false;
  int trials = 0;
  T e, c, pen = T(0);
  if (pr.M > 0) {
    const double* sp = sph + pr.sph;
    lm_cfg<NS, T, double>(rb, w, tt, z, lam, iters, o, failed, trials, sp, pr.M, 1, pr.sph_ld);
    ik_cost<NS>(rb, w, tt, z, &e);
    c = cfg_cost<NS, T, double>(rb, w, tt, z, sp, pr.M, 1, pr.sph_ld);
    WeightsT<T> wc = w;
    wc.w_pos = wc.w_rot = wc.sq_lim = wc.sq_curv = T(0);
    pen = cfg_cost<NS, T, double>(rb, wc, tt, z, sp, pr.M, 1, pr.sph_ld);
  } else {
    lm_ik<NS>(rb, w, tt, z, lam, iters, o, failed, trials);
    c = ik_cost<NS>(rb, w, tt, z, &e);
  }
  if (!tfinite(c) || !tfinite(e)) failed = true;
#pragma unroll
  for (int k = 0; k < NZ; ++k) z_out[k * B + b] = z[k];
  e_out[b] = e;
  pen_out[b] = pen;
  cost_out[b] = c;
  failed_out[b] = failed ? 1 : 0;
}

constexpr int kIkTile = 64;  // seeds per tile of the ragged IK stage 1

// One wave per tile of 64 consecutive seeds of one problem (tile0 of a problem in
// its table row's `pad`), so the problem's row, target and spheres are
// wave-uniform: scalar loads, and no wave mixes problems with and without
// clearance rows.
template <int NS, typename T, int OCC = 1>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC)))
    k_ik_stage1_rag(RobotT<T> rb, WeightsT<T> w, LMOpts<T> o, int64_t P, int64_t B, const IkProb* __restrict__ tp,
                    const double* __restrict__ task, const double* __restrict__ useed, const double* __restrict__ sph,
                    int iters, T lam0, T* __restrict__ z_out, T* __restrict__ e_out, T* __restrict__ pen_out,
                    T* __restrict__ cost_out, int32_t* __restrict__ failed_out, int n_tiles) {
  const int tile = __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  if (tile >= n_tiles) return;
  int64_t lo = 0, hi = P - 1;  // the last row whose first tile is <= tile
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (tp[mid].pad <= tile) lo = mid;
    else hi = mid - 1;
  }
  const IkProb pr = tp[lo];
  const int64_t s = (int64_t)(tile - pr.pad) * kIkTile + (threadIdx.x & 63);
  if (s >= pr.S) return;
  ik_rag_seed<NS, T>(rb, w, o, pr, pr.seed0 + s, s, B, task, useed, sph, iters, lam0, z_out, e_out, pen_out, cost_out,
                     failed_out);
}

// Persistent stage 1 of a ragged IK group over a work queue.  The items are tiles
// of kIkTile consecutive seeds of one problem, in the table's order (problems
// longest first, their tiles in seed order; tile0 of problem q in its table row's
// `pad`).  Each one-wave workgroup takes items from an atomic counter until the
// queue is empty, runs stage 1 on the tile's seeds (one lane per seed, the same
// per-seed code as k_ik_stage1_rag, so the same results), and counts the tile
// done for its problem; the wave that finishes a problem's last tile then runs
// that problem's SelectTop (n_final > 0).  No wave waits for another: the last
// arrival does the problem's remaining work, so every wave reaches the exit.
// q[0]: the queue head, q[1 + k]: tiles done of problem k (all zero on entry).

template <int NS, typename T, int OCC = 1>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC)))
    k_ik_stage1_q(RobotT<T> rb, WeightsT<T> w, LMOpts<T> o, int64_t P, int64_t B, const IkProb* __restrict__ tp,
                  const double* __restrict__ task, const double* __restrict__ useed, const double* __restrict__ sph,
                  int iters, T lam0, T* __restrict__ z_out, T* __restrict__ e_out, T* __restrict__ pen_out,
                  T* __restrict__ cost_out, int32_t* __restrict__ failed_out, int32_t* __restrict__ q, int n_final,
                  int Spad, int stage_pen, int stage_nz, T dup_eps, int32_t* __restrict__ sel) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const IkProb last = tp[P - 1];
  const int n_tiles = last.pad + (last.S + kIkTile - 1) / kIkTile;
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(&q[0], 1);
    item = __builtin_amdgcn_readfirstlane(item);  // lane 0's item, wave-uniform
    if (item >= n_tiles) break;
    // the problem of the tile: the last row whose first tile is <= item
    int64_t lo = 0, hi = P - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (tp[mid].pad <= item) lo = mid;
      else hi = mid - 1;
    }
    const IkProb pr = tp[lo];
    const int64_t s = (int64_t)(item - pr.pad) * kIkTile + lane;
    if (s < pr.S)
      ik_rag_seed<NS, T>(rb, w, o, pr, pr.seed0 + s, s, B, task, useed, sph, iters, lam0, z_out, e_out, pen_out,
                         cost_out, failed_out);
    if (n_final <= 0) continue;
    // publish this tile's results, then count it; the last tile's wave sees every
    // other tile's results after its own fence
    __threadfence();
    int done = 0;
    if (lane == 0) done = atomicAdd(&q[1 + lo], 1) + 1;
    done = __shfl(done, 0, 64);
    if (done != (pr.S + kIkTile - 1) / kIkTile) continue;
    __threadfence();
    SelRow row;
    row.S = pr.S;
    row.nz = 2 * NS;
    row.kbase = pr.seed0;
    row.zbase = pr.seed0;
    row.zsc = 1;
    select_top_one<T>(P, lo, pr.S, Spad, 2 * NS, stage_pen, stage_nz, z_out, B, 1, e_out, pen_out, failed_out, n_final,
                      dup_eps, &row, sel, smem);
    __syncthreads();  // the LDS of the selection is reused by the next problem
  }
}

__global__ void k_ik_selrows(int64_t P, int nz, const IkProb* __restrict__ tp, SelRow* __restrict__ rows) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  SelRow r;
  r.S = tp[q].S;
  r.nz = nz;
  r.kbase = tp[q].seed0;
  r.zbase = tp[q].seed0;
  r.zsc = 1;
  rows[q] = r;
}

template <int NS, typename T1>
__global__ void __launch_bounds__(256)
    k_ik_stage2_rag(RobotT<double> rb, WeightsT<double> w, LMOpts<double> o, int64_t P, int64_t B, int nf,
                    const IkProb* __restrict__ tp, const double* __restrict__ task, const double* __restrict__ sph,
                    const T1* __restrict__ z1, const int32_t* __restrict__ sel, int iters, double lam0,
                    double* __restrict__ z2, double* __restrict__ cost2, int32_t* __restrict__ failed2) {
  constexpr int NZ = 2 * NS;
  const int64_t B2 = P * (int64_t)nf;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B2) return;
  const int64_t p = b / nf;
  const int k = (int)(b % nf);
  const int s = sel[k * P + p];
  if (s < 0) {
#pragma unroll
    for (int m = 0; m < NZ; ++m) z2[m * B2 + b] = 0.0;
    cost2[b] = __builtin_nan("");
    failed2[b] = 1;
    return;
  }
  const IkProb pr = tp[p];
  double tt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) tt[c] = task[pr.task + c * pr.task_ld];
  double z[NZ];
#pragma unroll
  for (int m = 0; m < NZ; ++m) z[m] = (double)z1[m * B + pr.seed0 + s];
  double lam = lam0;
  bool failed = false;
  int trials = 0;
  double c;
  if (pr.M > 0) {
    const double* sp = sph + pr.sph;
    lm_cfg<NS, double, double>(rb, w, tt, z, lam, iters, o, failed, trials, sp, pr.M, 1, pr.sph_ld);
    c = cfg_cost<NS, double, double>(rb, w, tt, z, sp, pr.M, 1, pr.sph_ld);
  } else {
    lm_ik<NS>(rb, w, tt, z, lam, iters, o, failed, trials);
    c = ik_cost<NS>(rb, w, tt, z, (double*)nullptr);
  }
  if (!tfinite(c)) failed = true;
#pragma unroll
  for (int m = 0; m < NZ; ++m) z2[m * B2 + b] = z[m];
  cost2[b] = c;
  failed2[b] = failed ? 1 : 0;
}

// Argmin and FP64 assessment per problem.  Candidates: the nf stage-2 slots
// (sel != NULL) or every stage-1 seed of the problem.
template <int NS, typename TC>
__global__ void __launch_bounds__(256)
    k_ik_finalize_rag(RobotT<double> rb, int64_t P, int64_t Bc, int nf, const IkProb* __restrict__ tp,
                      const int32_t* __restrict__ sel, const TC* __restrict__ zc, const TC* __restrict__ costc,
                      const int32_t* __restrict__ failedc, const double* __restrict__ task,
                      const double* __restrict__ sph, int64_t err_ld, double* __restrict__ u_out,
                      double* __restrict__ err_out, int32_t* __restrict__ status_out) {
  constexpr int NZ = 2 * NS;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const IkProb pr = tp[p];
  const int nc = sel ? nf : pr.S;
  const int64_t c0 = sel ? p * nf : pr.seed0;
  int best = -1, best_seed = 0;
  double best_cost = 0.0;
  for (int k = 0; k < nc; ++k) {
    const int seed = sel ? sel[k * P + p] : k;
    const double c = (double)costc[c0 + k];
    if (seed < 0 || failedc[c0 + k] || !tfinite(c)) continue;
    if (best < 0 || c < best_cost || (c == best_cost && seed < best_seed)) {
      best = k;
      best_cost = c;
      best_seed = seed;
    }
  }
  double* uo = u_out + pr.out;
  const int64_t ei = pr.idx;
  if (best < 0) {
    const double nan = __builtin_nan("");
    for (int m = 0; m < 3 * NS; ++m) uo[m * pr.out_ld] = nan;
    err_out[ei] = err_out[err_ld + ei] = nan;
    status_out[ei] = CR_NONFINITE;
    return;
  }
  double z[NZ];
#pragma unroll
  for (int m = 0; m < NZ; ++m) z[m] = (double)zc[m * Bc + c0 + best];
  double tt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) tt[c] = task[pr.task + c * pr.task_ld];
  double Rc[9], pc[3];
  fk_tip<NS>(rb, z, Rc, pc);
  double dp[3] = {tt[3] - pc[0], tt[7] - pc[1], tt[11] - pc[2]};
  const double pos = sqrt(dot3(dp, dp));
  double Re[9], te[3];
  relative_pose(Rc, pc, tt, Re, te);
  double v[3] = {0.5 * (Re[7] - Re[5]), 0.5 * (Re[2] - Re[6]), 0.5 * (Re[3] - Re[1])};
  const double rot = atan2(sqrt(dot3(v, v)), 0.5 * (Re[0] + Re[4] + Re[8] - 1.0));
  double viol = -DBL_MAX, thx = -DBL_MAX;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double u[3];
    ab_to_u(z[2 * i], z[2 * i + 1], rb.rd[i], u);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      uo[(3 * i + j) * pr.out_ld] = u[j];
      viol = fmax(viol, fabs(u[j]) - rb.umaxd[i]);
    }
    thx = fmax(thx, sqrt(z[2 * i] * z[2 * i] + z[2 * i + 1] * z[2 * i + 1]) - rb.theta_maxd);
  }
  int32_t st = 0;
  if (viol > 1e-6 || thx > 0.0) st |= CR_LIMIT_VIOLATION;
  if (pr.M > 0 && penetrates<NS, double>(rb, z, sph + pr.sph, pr.M, pr.sph_ld)) st |= CR_COLLISION;
  if (!(pos <= 1e-3 && rot <= 3.14159265358979323846 / 180.0)) st |= CR_NOT_CONVERGED;
  if (st == 0) st = CR_SOLVED;
  err_out[ei] = pos;
  err_out[err_ld + ei] = rot;
  status_out[ei] = st;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t ik_workspace_layout(const cr_robot& rb, int64_t P, int32_t S, const cr_opts& o, cr_dtype dtype,
                           char* base, IkWorkspace* ws) {
  const size_t t1 = dtype == CR_F64 ? 8 : 4;
  const int64_t B = P * (int64_t)S;
  const int nz = (rb.extensible ? 3 : 2) * rb.n_seg;
  const int nf = o.n_final > 0 ? o.n_final : 0;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return base ? (void*)(base + at) : nullptr;
  };
  IkWorkspace w{};
  w.z1 = take(t1 * nz * B);
  w.e1 = take(t1 * B);
  w.pen1 = take(t1 * B);
  w.cost1 = take(t1 * B);
  w.failed1 = (int32_t*)take(4 * B);
  w.trials1 = (int32_t*)take(4 * B);
  w.sel = (int32_t*)take(4 * (size_t)(nf > 0 ? nf : 1) * P);
  w.z2 = (double*)take(8 * (size_t)nz * (nf > 0 ? nf : 1) * P);
  w.cost2 = (double*)take(8 * (size_t)(nf > 0 ? nf : 1) * P);
  w.failed2 = (int32_t*)take(4 * (size_t)(nf > 0 ? nf : 1) * P);
  if (ws) *ws = w;
  return off;
}


template <int NS, typename T>
static cr_status run_ik(const cr_robot& rb0, const cr_spheres* sp, int64_t P, const double* Tt, int32_t S,
                        const double* useed, const cr_weights& w0, const cr_opts& o, double* u_out, double* err_out,
                        int32_t* status_out, const IkWorkspace& ws, hipStream_t st) {
  const SphArgs sa{sp ? (const double*)sp->sph : nullptr, sp ? sp->ld : 0, sp ? sp->n_sph : 0,
                   sp ? sp->per_problem : 0, sp ? (const double*)sp->planes : nullptr, sp ? sp->plane_ld : 0,
                   sp ? sp->n_poly : 0, sp ? sp->n_planes : 0};
  // convex polytopes: the generic path with polytope rows (inextensible robots
  // without self contact; the API refuses the other combinations)
  if (sa.NPO > 0)
    return run_ik_gen<NS, T, false, false, true>(rb0, sa, P, Tt, S, useed, w0, o, u_out, err_out, status_out, ws, st);
  if constexpr (NS >= 3) {  // fewer than three segments have no non-adjacent pair
    if (rb0.self_collision && rb0.extensible)
      return run_ik_gen<NS, T, true, true>(rb0, sa, P, Tt, S, useed, w0, o, u_out, err_out, status_out, ws, st);
    if (rb0.self_collision)
      return run_ik_gen<NS, T, false, true>(rb0, sa, P, Tt, S, useed, w0, o, u_out, err_out, status_out, ws, st);
  }
  if (rb0.extensible)
    return run_ik_gen<NS, T, true, false>(rb0, sa, P, Tt, S, useed, w0, o, u_out, err_out, status_out, ws, st);
  RobotT<T> rb = robot_to<T>(rb0);
  WeightsT<T> w = weights_to<T>(w0);
  LMOpts<T> lo{o.ls_max, (T)o.lambda_min, (T)o.lambda_max};
  const int64_t B = P * (int64_t)S;
  const bool timed = timer_on();
  if (timed) timer_begin_call(st);
  if (sa.M > 0) {
    hipLaunchKernelGGL((k_ik_stage1_sph<NS, T>), dim3(blocks_for(P * (int64_t)((S + 63) / 64) * 64, 256)), dim3(256), 0,
                       st, rb, w, lo, P, (int)S,
                       Tt, useed, o.k_init, (T)o.lambda0, sa, (T*)ws.z1, (T*)ws.e1, (T*)ws.pen1, (T*)ws.cost1,
                       ws.failed1, ws.trials1);
  } else {
    auto launch = [&](int v) {
      const int occ = tune_occ(TK_IK_STAGE1, v);
#define CR_S1(O)                                                                                                   \
  hipLaunchKernelGGL((k_ik_stage1<NS, T, O>), dim3(blocks_for(B, 256)), dim3(256), 0, st, rb, w, lo, P, (int)S, Tt, \
                     useed, o.k_init, (T)o.lambda0, (T*)ws.z1, (T*)ws.e1, (T*)ws.pen1, (T*)ws.cost1, ws.failed1,   \
                     ws.trials1)
      if constexpr (sizeof(T) == 4) {
        if (occ == tune_occ(TK_IK_STAGE1, 1)) CR_S1(tune_occ(TK_IK_STAGE1, 1));
        else if (occ == tune_occ(TK_IK_STAGE1, 2)) CR_S1(tune_occ(TK_IK_STAGE1, 2));
        else CR_S1(1);
      } else {
        CR_S1(1);
      }
#undef CR_S1
    };
    int v = 0;
    bool done = false;
    if (sizeof(T) == 4) {
      cr_status rt = tune_choose(TK_IK_STAGE1, NS, CR_F32, B, st, launch, &v, &done);
      if (rt != CR_OK) return rt;
    }
    if (!done) launch(v);
  }
  cr_status rc = check_hip(hipGetLastError(), "k_ik_stage1");
  if (rc != CR_OK) return rc;
  if (timed) timer_mark(0, st);
  const bool two_stage = o.n_final > 0;
  RobotT<double> rbd = robot_to<double>(rb0);
  if (two_stage) {
    rc = launch_select(P, S, 2 * NS, ws.z1, ws.e1, ws.pen1, ws.failed1, o.n_final, o.dup_eps, ws.sel,
                       sizeof(T) == 8 ? CR_F64 : CR_F32, st);
    if (rc != CR_OK) return rc;
    if (timed) timer_mark(1, st);
    WeightsT<double> wd = weights_to<double>(w0);
    LMOpts<double> lod{o.ls_max, o.lambda_min, o.lambda_max};
    const int64_t B2 = P * (int64_t)o.n_final;
    if (sa.M > 0) {
      const int g2 = stage2_cfg_lanes(B2);
#define CR_S2C(GL)                                                                                                    \
  hipLaunchKernelGGL((k_ik_stage2<NS, T, true, false, false, GL>), dim3(blocks_for(stage2_threads(P, o.n_final, GL), 256)), \
                     dim3(256), 0, st, \
                     rbd, wd, lod, P, (int)S, (int)o.n_final, Tt, (const T*)ws.z1, ws.sel, o.k_final, o.lambda0, sa,  \
                     ws.z2, ws.cost2, ws.failed2)
      if (g2 == 4) CR_S2C(4);
      else if (g2 == 2) CR_S2C(2);
      else CR_S2C(1);
#undef CR_S2C
    } else {
      auto launch2 = [&](int g) {
#define CR_S2G(G)                                                                                                \
  hipLaunchKernelGGL((k_ik_stage2_grp<NS, T, G>), dim3(blocks_for(G * B2, 256)), dim3(256), 0, st, rbd, wd, lod, P, \
                     (int)S, (int)o.n_final, Tt, (const T*)ws.z1, ws.sel, o.k_final, o.lambda0, ws.z2, ws.cost2,   \
                     ws.failed2)
        if (g == 4) CR_S2G(4);
        else if (g == 2) CR_S2G(2);
        else CR_S2G(1);
#undef CR_S2G
      };
      // lanes per candidate: untuned, fill the 1024 SIMDs with one wave each where
      // the candidates allow, at most four
      int g = B2 * 4 <= kStage2Lanes ? 4 : (B2 * 2 <= kStage2Lanes ? 2 : 1);
      bool done = false;
      if (tune_enabled() || tune_forced() >= 0) {
        int v = 0;
        rc = tune_choose(TK_IK_STAGE2, NS, sizeof(T) == 8 ? CR_F64 : CR_F32, B2, st,
                         [&](int vv) { launch2(tune_occ(TK_IK_STAGE2, vv)); }, &v, &done);
        if (rc != CR_OK) return rc;
        if (!done && (tune_forced() >= 0 || tune_lookup(TK_IK_STAGE2, NS, sizeof(T) == 8 ? CR_F64 : CR_F32, B2) >= 0))
          g = tune_occ(TK_IK_STAGE2, v);
      }
      if (!done) launch2(g);
    }
    rc = check_hip(hipGetLastError(), "k_ik_stage2");
    if (rc != CR_OK) return rc;
    if (timed) timer_mark(2, st);
    hipLaunchKernelGGL((k_ik_finalize<NS, double>), dim3(blocks_for(P, 256)), dim3(256), 0, st, rbd, P,
                       (int)o.n_final, ws.sel, ws.z2, ws.cost2, ws.failed2, Tt, sa, u_out, err_out, status_out);
  } else {
    if (timed) {
      timer_mark(1, st);
      timer_mark(2, st);
    }
    hipLaunchKernelGGL((k_ik_finalize<NS, T>), dim3(blocks_for(P, 256)), dim3(256), 0, st, rbd, P, (int)S,
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

cr_status launch_solve_ik(const cr_robot& rb, const cr_spheres* sp, int64_t P, const double* Tt, int32_t S,
                          const double* useed, const cr_weights& w, const cr_opts& o, double* u_out, double* err_out,
                          int32_t* status_out, const IkWorkspace& ws, cr_dtype dtype, hipStream_t st) {
#define CR_IK_CASE(N)                                                                                            \
  case N:                                                                                                        \
    return dtype == CR_F64 ? run_ik<N, double>(rb, sp, P, Tt, S, useed, w, o, u_out, err_out, status_out, ws, st) \
                           : run_ik<N, float>(rb, sp, P, Tt, S, useed, w, o, u_out, err_out, status_out, ws, st);
  switch (rb.n_seg) {
    CR_IK_CASE(1)
    CR_IK_CASE(2)
    CR_IK_CASE(3)
    CR_IK_CASE(4)
    CR_IK_CASE(5)
    CR_IK_CASE(6)
    default:
      return fail(CR_EINVAL, "n_seg out of range");
  }
#undef CR_IK_CASE
}

// LDS plan of SelectTop for candidate counts up to S of nz coordinates: the
// padded count, whether penalties and coordinates are staged, and the bytes.
struct SelPlan {
  int Spad, stage_pen, stage_nz;
  size_t lds;
};

static SelPlan select_plan(int32_t S, int32_t nz, size_t tb) {
  SelPlan sp;
  sp.Spad = 1;
  while (sp.Spad < S) sp.Spad <<= 1;
  // stage the coordinates when every problem's fit in 32 KiB (nz == 0: per-row
  // counts unknown here, read from z)
  sp.stage_pen = select_lds(sp.Spad, 1, 0, tb) <= 64 * 1024 ? 1 : 0;
  sp.stage_nz = nz > 0 && (size_t)sp.Spad * nz * tb <= 32 * 1024 ? nz : 0;
  if (select_lds(sp.Spad, sp.stage_pen, sp.stage_nz, tb) > 64 * 1024) sp.stage_nz = 0;
  sp.lds = select_lds(sp.Spad, sp.stage_pen, sp.stage_nz, tb);
  return sp;
}

cr_status launch_select_strided(int64_t P, int32_t S, int32_t nz, const void* z, int64_t zs_m, int64_t zs_c,
                                const void* e, const void* pen, const int32_t* failed, int32_t n_final, double dup_eps,
                                int32_t* idx_out, cr_dtype dtype, hipStream_t st, const SelRow* rows) {
  const SelPlan sp = select_plan(S, nz, dtype == CR_F64 ? 8 : 4);
  const int Spad = sp.Spad, stage_pen = sp.stage_pen, stage_nz = sp.stage_nz;
  const size_t lds = sp.lds;
  if (P == 0) return CR_OK;
  if (dtype == CR_F64)
    hipLaunchKernelGGL((k_select<double>), dim3((unsigned)P), dim3(256), lds, st, P, (int)S, Spad, (int)nz, stage_pen,
                       stage_nz, (const double*)z, zs_m, zs_c, (const double*)e, (const double*)pen, failed, (int)n_final,
                       dup_eps, rows, idx_out);
  else
    hipLaunchKernelGGL((k_select<float>), dim3((unsigned)P), dim3(256), lds, st, P, (int)S, Spad, (int)nz, stage_pen,
                       stage_nz, (const float*)z, zs_m, zs_c, (const float*)e, (const float*)pen, failed, (int)n_final,
                       (float)dup_eps, rows, idx_out);
  return check_hip(hipGetLastError(), "k_select");
}

cr_status launch_select(int64_t P, int32_t S, int32_t nz, const void* z, const void* e, const void* pen,
                        const int32_t* failed, int32_t n_final, double dup_eps, int32_t* idx_out, cr_dtype dtype,
                        hipStream_t st) {
  return launch_select_strided(P, S, nz, z, P * (int64_t)S, 1, e, pen, failed, n_final, dup_eps, idx_out, dtype, st);
}

struct IkGroupWs {
  void *z1, *e1, *pen1, *cost1;
  int32_t *failed1, *sel;
  double *z2, *cost2;
  int32_t* failed2;
  IkProb* tp;
  SelRow* rows;
  int32_t* queue;  // persistent stage 1: queue head and tiles done per problem
};

static size_t ik_group_layout(int ns, int64_t P, int64_t B, int nf, cr_dtype dtype, char* base, IkGroupWs* w) {
  const size_t t1 = dtype == CR_F64 ? 8 : 4;
  const int nz = 2 * ns;
  const int64_t n2 = P * (nf > 0 ? nf : 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return base ? (void*)(base + at) : nullptr;
  };
  IkGroupWs x{};
  x.z1 = take(t1 * nz * B);
  x.e1 = take(t1 * B);
  x.pen1 = take(t1 * B);
  x.cost1 = take(t1 * B);
  x.failed1 = (int32_t*)take(4 * B);
  x.sel = (int32_t*)take(4 * n2);
  x.z2 = (double*)take(8 * nz * n2);
  x.cost2 = (double*)take(8 * n2);
  x.failed2 = (int32_t*)take(4 * n2);
  x.tp = (IkProb*)take(sizeof(IkProb) * P);
  x.rows = (SelRow*)take(sizeof(SelRow) * P);
  x.queue = (int32_t*)take(4 * (P + 1));
  if (w) *w = x;
  return off;
}

size_t ik_group_workspace_bytes(const cr_robot& rb, int64_t P, int64_t B, const cr_opts& o, cr_dtype dtype) {
  return ik_group_layout(rb.n_seg, P, B, o.n_final, dtype, nullptr, nullptr);
}

IkProb* ik_table_slot(const cr_robot& rb, int64_t P, int64_t B, const cr_opts& o, cr_dtype dtype, void* wsmem) {
  IkGroupWs w;
  ik_group_layout(rb.n_seg, P, B, o.n_final, dtype, (char*)wsmem, &w);
  return w.tp;
}

__global__ void k_zero_i32(int64_t n, int32_t* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

template <int NS, typename T>
static cr_status run_ik_group(const cr_robot& rb0, int64_t P, int64_t B, int Smax, const IkProb* tp,
                              const double* task, const double* useed, const double* sph, const cr_weights& w0,
                              const cr_opts& o, double* u_out, double* err_out, int64_t err_ld, int32_t* status_out,
                              const IkGroupWs& ws, bool persistent, int64_t n_tiles, hipStream_t st) {
  RobotT<T> rb = robot_to<T>(rb0);
  WeightsT<T> w = weights_to<T>(w0);
  LMOpts<T> lo{o.ls_max, (T)o.lambda_min, (T)o.lambda_max};
  RobotT<double> rbd = robot_to<double>(rb0);
  const SelPlan sp = select_plan(Smax, 2 * NS, sizeof(T));
  // persistent: enough one-wave workgroups to fill the chip several times over,
  // at most one per tile
  const unsigned qgrid = (unsigned)(n_tiles < 8192 ? n_tiles : 8192);
  auto launch = [&](int v) {
    const int occ = tune_occ(TK_IK_STAGE1_RAG, v);
#define CR_S1R(O)                                                                                                   \
  do {                                                                                                              \
    if (persistent) {                                                                                               \
      hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(P + 1, 256)), dim3(256), 0, st, P + 1, ws.queue);             \
      hipLaunchKernelGGL((k_ik_stage1_q<NS, T, O>), dim3(qgrid), dim3(64), sp.lds, st, rb, w, lo, P, B, tp, task,  \
                         useed, sph, o.k_init, (T)o.lambda0, (T*)ws.z1, (T*)ws.e1, (T*)ws.pen1, (T*)ws.cost1,     \
                         ws.failed1, ws.queue, o.n_final, sp.Spad, sp.stage_pen, sp.stage_nz, (T)o.dup_eps, ws.sel); \
    } else {                                                                                                        \
      hipLaunchKernelGGL((k_ik_stage1_rag<NS, T, O>), dim3(blocks_for(n_tiles * 64, 256)), dim3(256), 0, st, rb, w, \
                         lo, P, B, tp, task, useed, sph, o.k_init, (T)o.lambda0, (T*)ws.z1, (T*)ws.e1, (T*)ws.pen1, \
                         (T*)ws.cost1, ws.failed1, (int)n_tiles);                                                   \
    }                                                                                                               \
  } while (0)
    if constexpr (sizeof(T) == 4) {
      if (occ == tune_occ(TK_IK_STAGE1_RAG, 1)) CR_S1R(tune_occ(TK_IK_STAGE1_RAG, 1));
      else if (occ == tune_occ(TK_IK_STAGE1_RAG, 2)) CR_S1R(tune_occ(TK_IK_STAGE1_RAG, 2));
      else CR_S1R(1);
    } else {
      CR_S1R(1);
    }
#undef CR_S1R
  };
  int v = 0;
  bool done = false;
  if (sizeof(T) == 4) {
    cr_status rt = tune_choose(persistent ? TK_IK_STAGE1_Q : TK_IK_STAGE1_RAG, NS, CR_F32, B, st, launch, &v, &done);
    if (rt != CR_OK) return rt;
  }
  if (!done) launch(v);
  cr_status rc = check_hip(hipGetLastError(), "k_ik_stage1_rag");
  if (rc != CR_OK) return rc;
  if (o.n_final > 0) {
    const int nf = o.n_final;
    if (!persistent) {  // the persistent kernel has already selected
      hipLaunchKernelGGL(k_ik_selrows, dim3(blocks_for(P, 256)), dim3(256), 0, st, P, 2 * NS, tp, ws.rows);
      rc = launch_select_strided(P, Smax, 2 * NS, ws.z1, B, 1, ws.e1, ws.pen1, ws.failed1, nf, o.dup_eps, ws.sel,
                                 sizeof(T) == 8 ? CR_F64 : CR_F32, st, ws.rows);
      if (rc != CR_OK) return rc;
    }
    WeightsT<double> wd = weights_to<double>(w0);
    LMOpts<double> lod{o.ls_max, o.lambda_min, o.lambda_max};
    const int64_t B2 = P * (int64_t)nf;
    hipLaunchKernelGGL((k_ik_stage2_rag<NS, T>), dim3(blocks_for(B2, 256)), dim3(256), 0, st, rbd, wd, lod, P, B, nf,
                       tp, task, sph, (const T*)ws.z1, ws.sel, o.k_final, o.lambda0, ws.z2, ws.cost2, ws.failed2);
    hipLaunchKernelGGL((k_ik_finalize_rag<NS, double>), dim3(blocks_for(P, 256)), dim3(256), 0, st, rbd, P, B2, nf,
                       tp, ws.sel, ws.z2, ws.cost2, ws.failed2, task, sph, err_ld, u_out, err_out, status_out);
  } else {
    hipLaunchKernelGGL((k_ik_finalize_rag<NS, T>), dim3(blocks_for(P, 256)), dim3(256), 0, st, rbd, P, B, 0, tp,
                       (const int32_t*)nullptr, (const T*)ws.z1, (const T*)ws.cost1, ws.failed1, task, sph, err_ld,
                       u_out, err_out, status_out);
  }
  return check_hip(hipGetLastError(), "ragged IK");
}

cr_status launch_ik_group(const cr_robot& rb, int64_t P, int64_t B, int Smax, const IkProb* tp, const double* task,
                          const double* useed, const double* sph, const cr_weights& w, const cr_opts& o,
                          double* u_out, double* err_out, int64_t err_ld, int32_t* status_out, void* wsmem,
                          cr_dtype dtype, bool persistent, int64_t n_tiles, hipStream_t st) {
  IkGroupWs ws;
  ik_group_layout(rb.n_seg, P, B, o.n_final, dtype, (char*)wsmem, &ws);
  if (persistent && select_plan(Smax, 2 * rb.n_seg, dtype == CR_F64 ? 8 : 4).lds > 64 * 1024) persistent = false;
#define CR_IKG_CASE(N)                                                                                         \
  case N:                                                                                                      \
    return dtype == CR_F64 ? run_ik_group<N, double>(rb, P, B, Smax, tp, task, useed, sph, w, o, u_out, err_out, \
                                                     err_ld, status_out, ws, persistent, n_tiles, st)          \
                           : run_ik_group<N, float>(rb, P, B, Smax, tp, task, useed, sph, w, o, u_out, err_out,  \
                                                    err_ld, status_out, ws, persistent, n_tiles, st);
  switch (rb.n_seg) {
    CR_IKG_CASE(1)
    CR_IKG_CASE(2)
    CR_IKG_CASE(3)
    CR_IKG_CASE(4)
    CR_IKG_CASE(5)
    CR_IKG_CASE(6)
    default:
      return fail(CR_EINVAL, "n_seg out of range");
  }
#undef CR_IKG_CASE
}

}  // namespace crk
