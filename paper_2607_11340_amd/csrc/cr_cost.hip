// cr_cost.hip -- batched penalised cost (eq. 17) and its gradient by adjoint sweep.
//
//   k_cost_ik    one lane per seed (H = 0): pose + bounds + clearance
//   k_cost_traj  one workgroup per (problem, seed) trajectory, one lane per
//                waypoint (H + 1 <= 256): per-waypoint terms in registers,
//                neighbouring waypoints (smoothness, tip path length)
//                exchanged through LDS, spheres staged once in LDS
//
// The gradient never materialises a Jacobian: every cost term is turned into a
// force/torque at the tip or a force at a backbone point, and one reverse sweep
// over the stored twist columns maps them to dC/dz, then dC/du.
#include "cr_internal.h"

namespace crk {

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T s = T(0);
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

// EXT: extensible segments, the third coordinate e_i = mean_j u_ij per segment.
// POLY: convex polytopes (pl, NPO polytopes of F planes per problem or shared).
template <int NS, typename T, bool GRAD, bool EXT = false, bool SELF = false, bool POLY = false>
__global__ void __launch_bounds__(256)
    k_cost_ik(RobotT<T> rb, WeightsT<T> w, int64_t P, int S, const T* __restrict__ task, const T* __restrict__ sph,
              int64_t sld, int M, int per_problem, const T* __restrict__ u, T* __restrict__ cost, T* __restrict__ grad,
              const T* __restrict__ gscale, const T* __restrict__ pl, int64_t pld, int NPO, int F) {
  constexpr int NC = EXT ? 3 : 2, NZ = NC * NS;
  const int64_t B = P * (int64_t)S;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int64_t p = b / S;
  T z[NZ];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const T u0 = u[(3 * i) * B + b], u1 = u[(3 * i + 1) * B + b], u2 = u[(3 * i + 2) * B + b];
    u_to_ab(u0, u1, u2, rb.r[i], &z[NC * i], &z[NC * i + 1]);
    if constexpr (EXT) z[NC * i + 2] = (u0 + u1 + u2) * T(1.0 / 3.0);
  }
  T tt[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) tt[c] = task[c * P + p];
  Fwd<NS, T, EXT> f;
  const T* sp = sph ? sph + (per_problem ? p * M : 0) : nullptr;
  const PolyArgs<T> po{NPO > 0 ? pl + (per_problem ? p * NPO * F : 0) : nullptr, pld, NPO, F};
  T c = config_forward<NS, T, GRAD, T, T, EXT, SELF, POLY>(rb, w, z, sp, (sph && M > 0) ? M : 0, 1, sld, f, nullptr, po);
  T ft[3] = {T(0), T(0), T(0)}, tq[3] = {T(0), T(0), T(0)};
  c += pose_term<T, GRAD>(w, f.R, f.p, tt, ft, tq);
  cost[b] = c;
  if (GRAD) {
    T gz[NZ];
    config_reverse<NS, T, EXT>(f, ft, tq, gz);
    const T sc = gscale ? gscale[b] : T(1);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      T gu[3];
      gz_to_gu(gz[NC * i], gz[NC * i + 1], rb.r[i], gu);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if constexpr (EXT) gu[j] += gz[NC * i + 2] * T(1.0 / 3.0);  // de_i / du_ij = 1/3
        grad[(3 * i + j) * B + b] = sc * gu[j];
      }
    }
  }
}

template <int NS, typename T, bool GRAD>
__global__ void __launch_bounds__(256)
    k_cost_traj(RobotT<T> rb, WeightsT<T> w, int kind, int64_t P, int S, int H, const T* __restrict__ task,
                const T* __restrict__ sph, int64_t sld, int M, int per_problem, const T* __restrict__ u,
                T* __restrict__ cost, T* __restrict__ grad, const T* __restrict__ gscale) {
  constexpr int NZ = 2 * NS, NU = 3 * NS;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s_u = reinterpret_cast<T*>(smem_raw);  // zero-sum tendon displacements
  T* s_sph = s_u + (H + 1) * NU;
  T* s_p = s_sph + 4 * M;
  T* s_red = s_p + (H + 1) * 3;
  const int Tn = H + 1;
  const int64_t traj = blockIdx.x;
  const int64_t p = traj / S;
  const int64_t B = P * (int64_t)S * Tn;
  for (int i = threadIdx.x; i < 4 * M; i += blockDim.x) {
    const int m = i >> 2, cc = i & 3;
    s_sph[i] = sph[cc * sld + (per_problem ? p * M : 0) + m];
  }
  const int t = threadIdx.x;
  const bool act = t < Tn;
  const int64_t col = traj * Tn + t;
  T z[NZ];
  Fwd<NS, T> f;
  T cst = T(0);
  T ft[3] = {T(0), T(0), T(0)}, tq[3] = {T(0), T(0), T(0)};
  __syncthreads();
  if (act) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      u_to_ab(u[(3 * i) * B + col], u[(3 * i + 1) * B + col], u[(3 * i + 2) * B + col], rb.r[i], &z[2 * i],
              &z[2 * i + 1]);
      T ub[3];
      ab_to_u(z[2 * i], z[2 * i + 1], rb.r[i], ub);
#pragma unroll
      for (int j = 0; j < 3; ++j) s_u[t * NU + 3 * i + j] = ub[j];
    }
    cst = config_forward<NS, T, GRAD>(rb, w, z, s_sph, M, 4, 1, f);
    if (kind == CR_KIND_PATH) {
      T tt[12];
      const int64_t tc = p * Tn + t;
#pragma unroll
      for (int c = 0; c < 12; ++c) tt[c] = task[c * (P * Tn) + tc];
      cst += pose_term<T, GRAD>(w, f.R, f.p, tt, ft, tq);
    }
    s_p[3 * t] = f.p[0];
    s_p[3 * t + 1] = f.p[1];
    s_p[3 * t + 2] = f.p[2];
  }
  __syncthreads();
  if (act) {
    const T idt = T(1) / w.dt, idt2 = idt * idt;
    const T sqv = w.sq_vel, sqa = w.sq_acc, sql = w.sq_lim;
    T gu[NU];
    T cs = T(0);
#pragma unroll
    for (int m = 0; m < NU; ++m) gu[m] = T(0);
    // tendon velocity and acceleration (finite differences, Sec. IV-A): residual tau is
    // owned by lane tau for the cost; lane t gathers d/du_t from tau = t, t+1 (, t+2).
#pragma unroll
    for (int m = 0; m < NU; ++m) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int tau = t + k;
        if (tau >= 1 && tau <= H) {
          const T v = (s_u[tau * NU + m] - s_u[(tau - 1) * NU + m]) * idt;
          const T dv = k == 0 ? idt : -idt;
          const T rr = sqv * v;
          if (k == 0) cs += T(0.5) * rr * rr;
          if (GRAD) gu[m] += rr * sqv * dv;
          if (w.has_vmax) {
            const T viol = fabs(v) - w.v_max;
            if (viol > T(0)) {
              const T hr = sql * viol;
              if (k == 0) cs += T(0.5) * hr * hr;
              if (GRAD) gu[m] += hr * (v < T(0) ? -sql : sql) * dv;
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int tau = t + k;
        if (tau >= 2 && tau <= H) {
          const T a = (s_u[tau * NU + m] - T(2) * s_u[(tau - 1) * NU + m] + s_u[(tau - 2) * NU + m]) * idt2;
          const T da = k == 1 ? T(-2) * idt2 : idt2;
          const T rr = sqa * a;
          if (k == 0) cs += T(0.5) * rr * rr;
          if (GRAD) gu[m] += rr * sqa * da;
          if (w.has_amax) {
            const T viol = fabs(a) - w.a_max;
            if (viol > T(0)) {
              const T hr = sql * viol;
              if (k == 0) cs += T(0.5) * hr * hr;
              if (GRAD) gu[m] += hr * (a < T(0) ? -sql : sql) * da;
            }
          }
        }
      }
    }
    cst += cs;
    T gze[NZ];
#pragma unroll
    for (int k = 0; k < NZ; ++k) gze[k] = T(0);
    if (kind == CR_KIND_TRAJ) {
      // tip path length, eq. (11) squared: r_tau = sq_len (p_tau - p_{tau-1})
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (t >= 1) {
          const T rr = w.sq_len * (s_p[3 * t + c] - s_p[3 * (t - 1) + c]);
          cst += T(0.5) * rr * rr;
          ft[c] += rr * w.sq_len;
        }
        if (t + 1 <= H) ft[c] -= w.sq_len * w.sq_len * (s_p[3 * (t + 1) + c] - s_p[3 * t + c]);
      }
      // endpoint equalities, penalised (eq. 17)
      if (t == 0 || t == H) {
        const int off = t == 0 ? 0 : NU;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          T za, zb;
          u_to_ab(task[(off + 3 * i) * P + p], task[(off + 3 * i + 1) * P + p], task[(off + 3 * i + 2) * P + p],
                  rb.r[i], &za, &zb);
          const T sqe = w.sq_eq;
          const T ra = sqe * (z[2 * i] - za), rb2 = sqe * (z[2 * i + 1] - zb);
          cst += T(0.5) * (ra * ra + rb2 * rb2);
          gze[2 * i] += sqe * ra;
          gze[2 * i + 1] += sqe * rb2;
        }
      }
    }
    if (GRAD) {
      T gz[NZ];
      config_reverse<NS>(f, ft, tq, gz);
      const T sc = gscale ? gscale[traj] : T(1);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        T sa = T(0), sb = T(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          T ja, jb;
          lift_row(j, rb.r[i], &ja, &jb);
          sa += gu[3 * i + j] * ja;
          sb += gu[3 * i + j] * jb;
        }
        const T ga = gz[2 * i] + gze[2 * i] + sa, gb = gz[2 * i + 1] + gze[2 * i + 1] + sb;
        T go[3];
        gz_to_gu(ga, gb, rb.r[i], go);
#pragma unroll
        for (int j = 0; j < 3; ++j) grad[(3 * i + j) * B + col] = sc * go[j];
      }
    }
  }
  const T total = block_sum(cst, s_red);
  if (threadIdx.x == 0) cost[traj] = total;
}

template <int NS, typename T>
static cr_status run_cost(int kind, const cr_robot& rb0, const cr_spheres* sp, const cr_weights& w0, int64_t P, int H,
                          int S, const void* task, const void* u, void* cost, void* grad, const void* gscale,
                          hipStream_t st) {
  RobotT<T> rb = robot_to<T>(rb0);
  WeightsT<T> w = weights_to<T>(w0);
  const int M = sp ? sp->n_sph : 0;
  const T* sph = M > 0 ? (const T*)sp->sph : nullptr;
  const int64_t sld = M > 0 ? sp->ld : 0;
  const int NPO = sp ? sp->n_poly : 0;
  const int ppb = (M > 0 || NPO > 0) ? sp->per_problem : 0;
  const T* pl = NPO > 0 ? (const T*)sp->planes : nullptr;
  const int64_t pld = NPO > 0 ? sp->plane_ld : 0;
  const int F = NPO > 0 ? sp->n_planes : 0;
  const int64_t B = P * (int64_t)S;
  if (B == 0) return CR_OK;
  if (kind == CR_KIND_IK) {
    const unsigned nb = (unsigned)((B + 255) / 256);
#define CR_COST_IK(G, E, SF, PO)                                                                                   \
  hipLaunchKernelGGL((k_cost_ik<NS, T, G, E, SF, PO>), dim3(nb), dim3(256), 0, st, rb, w, P, S, (const T*)task, sph, \
                     sld, M, ppb, (const T*)u, (T*)cost, G ? (T*)grad : (T*)nullptr,                                 \
                     G ? (const T*)gscale : (const T*)nullptr, pl, pld, NPO, F)
#define CR_COST_IK2(E, SF)              \
  do {                                  \
    if (grad)                           \
      CR_COST_IK(true, E, SF, false);   \
    else                                \
      CR_COST_IK(false, E, SF, false);  \
  } while (0)
    const bool self = rb0.self_collision && NS >= 3;
    if (NPO > 0) {  // convex polytopes: inextensible robots without self contact
      if (grad) CR_COST_IK(true, false, false, true);
      else CR_COST_IK(false, false, false, true);
    } else if (rb0.extensible && self) CR_COST_IK2(true, true);
    else if (rb0.extensible) CR_COST_IK2(true, false);
    else if (self) CR_COST_IK2(false, true);
    else CR_COST_IK2(false, false);
#undef CR_COST_IK2
#undef CR_COST_IK
    return check_hip(hipGetLastError(), "k_cost_ik");
  }
  const int Tn = H + 1;
  const int threads = ((Tn + 63) / 64) * 64;
  const size_t lds = sizeof(T) * (size_t)(Tn * 3 * NS + 4 * M + Tn * 3 + 8);
  if (grad)
    hipLaunchKernelGGL((k_cost_traj<NS, T, true>), dim3((unsigned)B), dim3(threads), lds, st, rb, w, kind, P, S, H,
                       (const T*)task, sph, sld, M, ppb, (const T*)u, (T*)cost, (T*)grad, (const T*)gscale);
  else
    hipLaunchKernelGGL((k_cost_traj<NS, T, false>), dim3((unsigned)B), dim3(threads), lds, st, rb, w, kind, P, S, H,
                       (const T*)task, sph, sld, M, ppb, (const T*)u, (T*)cost, (T*)nullptr, (const T*)nullptr);
  return check_hip(hipGetLastError(), "k_cost_traj");
}

cr_status launch_cost_grad(int kind, const cr_robot& rb, const cr_spheres* sp, const cr_weights& w, int64_t P, int H,
                           int S, const void* task, const void* u, void* cost, void* grad, const void* gscale,
                           cr_dtype dtype, hipStream_t st) {
#define CR_COST_CASE(N)                                                                                   \
  case N:                                                                                                 \
    return dtype == CR_F64 ? run_cost<N, double>(kind, rb, sp, w, P, H, S, task, u, cost, grad, gscale, st) \
                           : run_cost<N, float>(kind, rb, sp, w, P, H, S, task, u, cost, grad, gscale, st);
  switch (rb.n_seg) {
    CR_COST_CASE(1)
    CR_COST_CASE(2)
    CR_COST_CASE(3)
    CR_COST_CASE(4)
    CR_COST_CASE(5)
    CR_COST_CASE(6)
    default:
      return fail(CR_EINVAL, "n_seg out of range");
  }
#undef CR_COST_CASE
}

}  // namespace crk
