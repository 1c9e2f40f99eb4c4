// cr_calib.hip -- calibration kernels for the roofline accounting: vector-ALU
// loops with a known instruction mix, so that the issue rate the hardware reaches
// (and what the SQ_INSTS_VALU* counters count) can be measured directly.
//
// Each lane runs `iters` rounds over 16 independent chains, so that latency is
// hidden and the SIMD issue rate bounds the loop:
//   kind 0: one v_fma_f32 per chain and round (16 FMA per round);
//   kind 1: one v_rcp_f32 per chain and round (16 transcendental per round);
//   kind 2: one v_fma_f32 per chain plus one v_rcp_f32 on every fourth chain
//           (16 FMA + 4 transcendental per round);
//   kind 3: one v_fma_f64 per chain and round (16 FP64 FMA per round);
//   kind 4: one v_add_f32 per chain and round;
//   kind 5: one v_mul_f32 per chain and round;
//   kind 6: one v_fma_f32 per chain and round over 32 chains (32 per round);
//   kind 7: 10 v_fma_f32, 4 v_mul_f32 and 2 v_add_f32 per round (the
//           FMA : MUL : ADD proportions of the IK stage-1 kernel);
//   kind 8: as kind 0 with only lanes 0..31 of every wave active;
//   kind 9: as kind 0 with only lanes 0..15 of every wave active.
// The result of every chain reaches memory, so nothing is removed by the compiler.
#include "cr_internal.h"

namespace crk {

template <int KIND>
__global__ void __launch_bounds__(256) k_calib_valu(int iters, float a, float b, float* __restrict__ out) {
  constexpr int kCalibChains = KIND == 6 ? 32 : 16;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (KIND == 8 || KIND == 9) {
    if ((threadIdx.x & 63) >= (KIND == 8 ? 32 : 16)) {
      out[g] = 0.0f;
      return;
    }
  }
  if constexpr (KIND == 3) {
    double x[kCalibChains];
#pragma unroll
    for (int c = 0; c < kCalibChains; ++c) x[c] = 1e-3 * (double)threadIdx.x + (double)c;
    const double ad = (double)a, bd = (double)b;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kCalibChains; ++c) x[c] = fma(x[c], ad, bd);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kCalibChains; ++c) s += x[c];
    out[g] = (float)s;
  } else {
    float x[kCalibChains];
#pragma unroll
    for (int c = 0; c < kCalibChains; ++c) x[c] = 1e-3f * (float)threadIdx.x + (float)c + 1.0f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kCalibChains; ++c) {
        if constexpr (KIND == 0 || KIND == 6 || KIND == 8 || KIND == 9) {
          x[c] = fmaf(x[c], a, b);
        } else if constexpr (KIND == 1) {
          x[c] = __builtin_amdgcn_rcpf(x[c]);
        } else if constexpr (KIND == 2) {
          x[c] = fmaf(x[c], a, b);
          if (c % 4 == 0) x[c] = __builtin_amdgcn_rcpf(x[c]);
        } else if constexpr (KIND == 4) {
          x[c] = x[c] + b;
        } else if constexpr (KIND == 5) {
          x[c] = x[c] * a;
        } else {
          x[c] = c < 10 ? fmaf(x[c], a, b) : (c < 14 ? x[c] * a : x[c] + b);
        }
      }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kCalibChains; ++c) s += x[c];
    out[g] = s;
  }
}

}  // namespace crk

using namespace crk;

// Launches `blocks` workgroups of 256 lanes of calibration loop `kind` (0..9)
// with `iters` rounds; out [device] receives blocks * 256 floats.
extern "C" cr_status cr_calib_valu(int32_t kind, int64_t blocks, int32_t iters, float* out, hipStream_t stream) {
  if (kind < 0 || kind > 9) return fail(CR_EINVAL, "kind %d not in 0..9", kind);
  if (blocks < 1 || blocks > (1 << 20) || iters < 1) return fail(CR_EINVAL, "blocks / iters out of range");
  if (!out) return fail(CR_EINVAL, "out is NULL");
  const float a = 0.999f, b = 1e-4f;
  const dim3 grid((unsigned)blocks), block(256);
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_calib_valu<0>, grid, block, 0, stream, iters, a, b, out);
      break;
    case 1:
      hipLaunchKernelGGL(k_calib_valu<1>, grid, block, 0, stream, iters, a, b, out);
      break;
    case 2:
      hipLaunchKernelGGL(k_calib_valu<2>, grid, block, 0, stream, iters, a, b, out);
      break;
    case 3:
      hipLaunchKernelGGL(k_calib_valu<3>, grid, block, 0, stream, iters, a, b, out);
      break;
    case 4:
      hipLaunchKernelGGL(k_calib_valu<4>, grid, block, 0, stream, iters, a, b, out);
      break;
    case 5:
      hipLaunchKernelGGL(k_calib_valu<5>, grid, block, 0, stream, iters, a, b, out);
      break;
    case 6:
      hipLaunchKernelGGL(k_calib_valu<6>, grid, block, 0, stream, iters, a, b, out);
      break;
    case 8:
      hipLaunchKernelGGL(k_calib_valu<8>, grid, block, 0, stream, iters, a, b, out);
      break;
    case 9:
      hipLaunchKernelGGL(k_calib_valu<9>, grid, block, 0, stream, iters, a, b, out);
      break;
    default:
      hipLaunchKernelGGL(k_calib_valu<7>, grid, block, 0, stream, iters, a, b, out);
      break;
  }
  return check_hip(hipGetLastError(), "k_calib_valu");
}
