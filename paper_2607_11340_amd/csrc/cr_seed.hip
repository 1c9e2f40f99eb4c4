// cr_seed.hip -- SampleSeeds of Algorithm 1 on the device (Sec. IV-B: seeds
// inside the bounds, seeds that collide at once drawn again).
//
//   k_sample_seeds  one lane per (problem, seed): draws from a Philox4x64-10
//                   stream keyed by (key, problem, seed, attempt), so the seed
//                   of (p, s) does not depend on the launch shape; the collision
//                   test is the FP64 one of the final assessment.
#include "cr_internal.h"

namespace crk {

// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011): per round, words 0
// and 2 are multiplied by the round multipliers into 128-bit products whose high
// halves are mixed with words 1 and 3 and the key; the key advances by the two
// Weyl increments between rounds.
struct Philox4x64 {
  uint64_t w[4];
};

__device__ __forceinline__ Philox4x64 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                                    uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  return Philox4x64{{c0, c1, c2, c3}};
}

// The uniform stream of one (problem, seed, attempt): U_j is word j mod 4 of
// the block at counter (j div 4, attempt, seed, problem), its top 53 bits times
// 2^-53.  Blocks are generated four uniforms at a time.
struct SeedStream {
  uint64_t k0, k1, a, s, p;
  uint64_t j = 0;
  Philox4x64 blk;
  __device__ double next() {
    if ((j & 3) == 0) blk = philox4x64_10(j >> 2, a, s, p, k0, k1);
    const uint64_t x = blk.w[j & 3];
    ++j;
    return (double)(x >> 11) * 0x1.0p-53;
  }
};

template <int NS, bool EXT, bool SELF>
__global__ void __launch_bounds__(256)
    k_sample_seeds(RobotT<double> rb, int64_t P, int S, uint64_t key0, uint64_t key1, int max_attempts,
                   const double* __restrict__ sph, int M, int per_problem, int64_t ld, double* __restrict__ u_out,
                   int32_t* __restrict__ attempts_out) {
  constexpr int NC = EXT ? 3 : 2;
  const int64_t B = P * (int64_t)S;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int64_t p = b / S;
  const int s = (int)(b - p * S);
  const double* sp = M > 0 ? sph + (per_problem ? p * M : 0) : nullptr;
  // cos and sin of the tendon angles 0, 2 pi / 3, 4 pi / 3 (eq. 4)
  const double ca[3] = {1.0, -0.5, -0.5}, sa[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
  double u[3 * NS], z[NC * NS];
  int a = 0;
  bool hit = false;
  for (;; ++a) {
    SeedStream rs{key0, key1, (uint64_t)a, (uint64_t)s, (uint64_t)p};
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const double bnd = rb.umax[i];
      double ub[3] = {0.0, 0.0, 0.0}, worst = 0.0, th = 0.0;
      bool ok = false;
      for (int tries = 0; tries < kSeedTriples && !ok; ++tries) {
        double x[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) x[k] = bnd * (2.0 * rs.next() - 1.0);
        const double mean = (x[0] + x[1] + x[2]) / 3.0;
        worst = 0.0;
        double pc = 0.0, ps = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          ub[k] = x[k] - mean;
          worst = fmax(worst, fabs(ub[k]));
          pc += ub[k] * ca[k];
          ps += ub[k] * sa[k];
        }
        th = sqrt(pc * pc + ps * ps) / (1.5 * rb.r[i]);
        ok = worst <= bnd && th <= rb.theta_max;
      }
      if (!ok) {  // no triple inside the bounds: the last one scaled onto them
        const double f = fmin(worst > 0.0 ? bnd / worst : 1.0, th > 0.0 ? rb.theta_max / th : 1.0);
#pragma unroll
        for (int k = 0; k < 3; ++k) ub[k] *= f;
      }
      double e = 0.0;
      if constexpr (EXT) e = (rb.Lmid[i] - rb.Lhalf[i] - rb.L[i]) + 2.0 * rb.Lhalf[i] * rs.next();
#pragma unroll
      for (int k = 0; k < 3; ++k) u[3 * i + k] = ub[k] + e;
      u_to_ab(ub[0], ub[1], ub[2], rb.r[i], &z[NC * i], &z[NC * i + 1]);
      if constexpr (EXT) z[NC * i + 2] = e;
    }
    hit = (M > 0 || SELF) && penetrates<NS, double, EXT, SELF>(rb, z, sp, M, ld);
    if (!hit || a + 1 >= max_attempts) break;
  }
#pragma unroll
  for (int m = 0; m < 3 * NS; ++m) u_out[m * B + b] = u[m];
  if (attempts_out) attempts_out[b] = hit ? -(a + 1) : a + 1;
}

template <int NS>
static cr_status run_sample(const cr_robot& rb0, const cr_spheres* sp, int64_t P, int32_t S, uint64_t k0, uint64_t k1,
                            int32_t max_attempts, double* u_out, int32_t* att, hipStream_t st) {
  const RobotT<double> rb = robot_to<double>(rb0);
  const int M = sp ? sp->n_sph : 0;
  const double* sph = M > 0 ? (const double*)sp->sph : nullptr;
  const int ppb = M > 0 ? sp->per_problem : 0;
  const int64_t ld = M > 0 ? sp->ld : 0;
  const int64_t B = P * (int64_t)S;
  const dim3 grid((unsigned)((B + 255) / 256)), block(256);
#define CR_SEED(E, SF)                                                                                            \
  hipLaunchKernelGGL((k_sample_seeds<NS, E, SF>), grid, block, 0, st, rb, P, (int)S, k0, k1, (int)max_attempts, sph, \
                     M, ppb, ld, u_out, att)
  const bool ext = rb0.extensible != 0;
  if constexpr (NS >= 3) {
    if (rb0.self_collision) {
      if (ext) CR_SEED(true, true);
      else CR_SEED(false, true);
      return check_hip(hipGetLastError(), "k_sample_seeds");
    }
  }
  if (ext) CR_SEED(true, false);
  else CR_SEED(false, false);
#undef CR_SEED
  return check_hip(hipGetLastError(), "k_sample_seeds");
}

cr_status launch_sample_seeds(const cr_robot& rb, const cr_spheres* sp, int64_t P, int32_t S, uint64_t k0,
                              uint64_t k1, int32_t max_attempts, double* u_out, int32_t* attempts_out,
                              hipStream_t st) {
  if (P * (int64_t)S == 0) return CR_OK;
  switch (rb.n_seg) {
    case 1: return run_sample<1>(rb, sp, P, S, k0, k1, max_attempts, u_out, attempts_out, st);
    case 2: return run_sample<2>(rb, sp, P, S, k0, k1, max_attempts, u_out, attempts_out, st);
    case 3: return run_sample<3>(rb, sp, P, S, k0, k1, max_attempts, u_out, attempts_out, st);
    case 4: return run_sample<4>(rb, sp, P, S, k0, k1, max_attempts, u_out, attempts_out, st);
    case 5: return run_sample<5>(rb, sp, P, S, k0, k1, max_attempts, u_out, attempts_out, st);
    case 6: return run_sample<6>(rb, sp, P, S, k0, k1, max_attempts, u_out, attempts_out, st);
  }
  return fail(CR_EINVAL, "n_seg out of range");
}

}  // namespace crk
