// cr_fk.hip -- batched forward kinematics (Sec. III-A eq. 1-3, Sec. III-B eq. 4).
//
// One lane per configuration; loads and stores are structure-of-arrays with the
// batch index fastest, so every component access of a wavefront is one
// coalesced 256 B (FP32) or 512 B (FP64) transaction.  The kernel is HBM bound:
// 3n values in, 3n + 12n (+3nK) values out per configuration.
#include "cr_internal.h"

namespace crk {

// One Newton-Schulz step toward the nearest rotation, R <- R (3 I - R^T R) / 2,
// in FP64: squares the orthogonality error of an FP32 chained product.
__device__ __forceinline__ void reorthonormalize(double* R) {
  double M[9], Q[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = R[i] * R[j] + R[3 + i] * R[3 + j] + R[6 + i] * R[6 + j];
      M[3 * i + j] = (i == j ? 3.0 : 0.0) - s;
    }
  mm3(R, M, Q);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = 0.5 * Q[k];
}

template <int NS, typename T>
__global__ void __launch_bounds__(256)
    k_fk(RobotT<T> rb, int64_t B, const T* __restrict__ u, int64_t ld, T* __restrict__ arc,
         T* __restrict__ frames, T* __restrict__ pts) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  T Rc[9], pc[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = (k % 4 == 0) ? T(1) : T(0);
  pc[0] = pc[1] = pc[2] = T(0);
  const int K = rb.K;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    T a, bb;
    const T u0 = u[(3 * i) * ld + b], u1 = u[(3 * i + 1) * ld + b], u2 = u[(3 * i + 2) * ld + b];
    u_to_ab(u0, u1, u2, rb.r[i], &a, &bb);
    // extensible segments: the common mode of the three tendons is the change of length
    const T Li = rb.ext ? rb.L[i] + (u0 + u1 + u2) * T(1.0 / 3.0) : rb.L[i];
    T s = a * a + bb * bb;
    if (arc) {
      T th = tsqrt(s);
      T ph = th > T(0) ? tatan2(bb, a) : T(0);
      if (ph < T(0)) ph += T(6.28318530717958647692);
      arc[(3 * i) * ld + b] = th / Li;
      arc[(3 * i + 1) * ld + b] = ph;
      arc[(3 * i + 2) * ld + b] = Li;
    }
    if (pts) {
      for (int k = 1; k <= K; ++k) {
        T sg = T(k) / T(K);
        ArcCoef<T> ck = arc_coef<T, false>(sg * sg * s);
        T Rk[9], dk[3], q[3];
        seg_R_d(sg * a, sg * bb, sg * Li, ck, Rk, dk);
        mv3(Rc, dk, q);
        const int64_t c0 = 3 * (i * K + k - 1);
        pts[c0 * ld + b] = pc[0] + q[0];
        pts[(c0 + 1) * ld + b] = pc[1] + q[1];
        pts[(c0 + 2) * ld + b] = pc[2] + q[2];
      }
    }
    ArcCoef<T> c = arc_coef<T, false>(s);
    T Ri[9], di[3], q[3], Rn[9];
    seg_R_d(a, bb, Li, c, Ri, di);
    mv3(Rc, di, q);
    pc[0] += q[0];
    pc[1] += q[1];
    pc[2] += q[2];
    mm3(Rc, Ri, Rn);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = Rn[k];
    if (frames) {
      double Ro[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Ro[k] = (double)Rc[k];
      if (sizeof(T) == 4) reorthonormalize(Ro);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) frames[(12 * i + 4 * r + cc) * ld + b] = (T)Ro[3 * r + cc];
        frames[(12 * i + 4 * r + 3) * ld + b] = pc[r];
      }
    }
  }
}

template <int NS, typename T>
static cr_status run_fk(const cr_robot& rb0, int64_t B, const void* u, int64_t ld, void* arc, void* frames, void* pts,
                        hipStream_t st) {
  RobotT<T> rb = robot_to<T>(rb0);
  if (B == 0) return CR_OK;
  hipLaunchKernelGGL((k_fk<NS, T>), dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, rb, B, (const T*)u, ld,
                     (T*)arc, (T*)frames, (T*)pts);
  return check_hip(hipGetLastError(), "k_fk");
}

cr_status launch_fk(const cr_robot& rb, int64_t B, const void* u, int64_t ld, void* arc, void* frames, void* pts,
                    cr_dtype dtype, hipStream_t st) {
#define CR_FK_CASE(N)                                                               \
  case N:                                                                           \
    return dtype == CR_F64 ? run_fk<N, double>(rb, B, u, ld, arc, frames, pts, st) \
                           : run_fk<N, float>(rb, B, u, ld, arc, frames, pts, st);
  switch (rb.n_seg) {
    CR_FK_CASE(1)
    CR_FK_CASE(2)
    CR_FK_CASE(3)
    CR_FK_CASE(4)
    CR_FK_CASE(5)
    CR_FK_CASE(6)
    default:
      return fail(CR_EINVAL, "n_seg out of range");
  }
#undef CR_FK_CASE
}

}  // namespace crk
