// cr_traj.hip -- path following (eq. 16) and trajectory planning (eq. 11-15):
// Levenberg-Marquardt over whole trajectories inside the two-stage template.
//
// Per LM iteration three kernels run over every trajectory (problem x seed):
//   k_traj_build   one workgroup per trajectory, one lane per waypoint: each lane
//                  forms its Gauss-Newton block (pose, bounds, clearance rows)
//                  and, through LDS, the smoothness and path-length couplings to
//                  waypoints t-1 and t-2; writes the block rows of
//                  H = J^T J (diagonal, first and second sub-diagonal blocks) and g.
//   k_traj_solve   NZ lanes per trajectory, one per row of the 2n x 2n blocks,
//                  several trajectories per wave: damping, block Cholesky of the
//                  block-pentadiagonal H + lambda D (the exact banded factor),
//                  forward and backward substitution, g.delta.
//   k_traj_search  one workgroup per trajectory: backtracking line search; the
//                  trial cost is block-reduced, so accept/reject is uniform per
//                  workgroup; updates z and lambda.
// Per trajectory and waypoint the workspace holds one record (struct Rec) and z
// is stored trajectory-major, waypoint, coordinate: [traj][t][k].  A trajectory's
// flag is 0 while it iterates, 1 once its cost is not finite (never selected) and
// 2 once a step was rejected at the largest damping: z and lambda then repeat in
// every later iteration, so its kernels skip it with the result unchanged.
#include <float.h>

#include "cr_internal.h"

namespace crk {

template <typename T>
struct TrajArgs {
  int kind;                 // CR_KIND_PATH or CR_KIND_TRAJ
  int64_t P;                // problems in the launch
  int nf;                   // 0: stage 1, S of each problem's trajectories; > 0: nf per problem (stage 2)
  int Tmax;                 // largest horizon + 1 of the launch
  const TrajProb* tp;       // one row per problem
  const double* task;       // PATH: reference poses; TRAJ: start and goal actuations (see TrajProb)
  const double* sph;        // spheres (see TrajProb) or NULL
};

// What a workgroup (or lane group) needs of the trajectory it works on.
struct TrajCtx {
  TrajProb pr;
  int64_t q;   // problem
  int s;       // trajectory of the problem (seed, or stage-2 slot)
  int64_t wp;  // first waypoint configuration of the trajectory in Z and the records
};

template <typename T>
__device__ __forceinline__ TrajCtx traj_ctx(const TrajArgs<T>& ta, int64_t traj) {
  TrajCtx cx;
  if (ta.nf > 0) {
    cx.q = traj / ta.nf;
    cx.pr = ta.tp[cx.q];
    cx.s = (int)(traj - cx.q * ta.nf);
    cx.wp = ta.nf * cx.pr.tn0 + (int64_t)cx.s * cx.pr.Tn;
  } else {
    int64_t lo = 0, hi = ta.P - 1;  // last problem whose first trajectory is <= traj
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (ta.tp[mid].traj0 <= traj) lo = mid;
      else hi = mid - 1;
    }
    cx.q = lo;
    cx.pr = ta.tp[lo];
    cx.s = (int)(traj - cx.pr.traj0);
    cx.wp = cx.pr.wp0 + (int64_t)cx.s * cx.pr.Tn;
  }
  return cx;
}

// Per-waypoint record of the normal equations and of their factor.  The block
// solve streams these records through HBM twice per LM iteration, so the build
// stores only what is not zero or repeated, and the solve keeps row a of every
// block on lane a.  Inputs, written by the build and read once by the forward
// pass:
//   OHI: H_tt, lower triangle packed by rows (element (i, j), j <= i, at
//        i (i + 1) / 2 + j; the upper triangle is never read)
//   OBS, OCS: the smoothness couplings, 2 x 2 symmetric blocks on the diagonal,
//        (aa, ab, bb) per segment: H_{t,t-2} is exactly that, and so is H_{t,t-1}
//        for path following
//   OB:  trajectories only: H_{t,t-1} in full (the tip path-length term couples
//        every coordinate of t with every one of t - 1), row-major
//   OG:  g_t
// Factor, written by the forward pass and read by the backward pass:
//   OL:  L_tt, lower triangle packed by columns (column j from
//        j NZ - j (j - 1) / 2, rows j .. NZ - 1: the backward pass reads a column
//        per lane)
//   OB:  L_{t,t-1}, row-major (element (i, j) at i NZ + j: the forward pass
//        writes a row per lane as NZ consecutive values)
//   OY:  y_t, then delta_t
// L_{t,t-2} = H_{t,t-2} L_{t-2,t-2}^-T is not stored: the backward pass forms
// L_{t,t-2}^T delta_t as L_{t-2,t-2}^-1 (H_{t,t-2}^T delta_t) from the segment
// blocks, a triangular solve instead of a block read and write through HBM.
__host__ __device__ constexpr int rec_up4(int x) { return (x + 3) & ~3; }
__host__ __device__ constexpr int rec_size(int ns) {
  return 2 * rec_up4(2 * ns * (2 * ns + 1) / 2) + (2 * ns) * (2 * ns) + 2 * rec_up4(2 * ns) + 2 * rec_up4(3 * ns);
}
template <int NS>
struct Rec {
  static constexpr int NZ = 2 * NS, NP = NZ * (NZ + 1) / 2;
  static constexpr int OL = 0, OB = rec_up4(NP), OY = OB + NZ * NZ, OG = OY + rec_up4(NZ),
                       OHI = OG + rec_up4(NZ), OBS = OHI + rec_up4(NP), OCS = OBS + rec_up4(3 * NS),
                       SIZE = OCS + rec_up4(3 * NS);
  // with a 256-byte aligned workspace every record and block starts on a 16-byte
  // boundary in FP32 and FP64; a row of OB is 16-byte aligned when NZ is a
  // multiple of 4 or in FP64, else 8-byte aligned
  static_assert(SIZE % 4 == 0 && OB % 4 == 0 && OY % 4 == 0 && OG % 4 == 0,
                "record blocks must be 16-byte aligned");
  static_assert(SIZE == rec_size(NS), "rec_size must follow the layout");
  // first value of column j of L_tt in OL
  static __device__ __forceinline__ int lcol(int j) { return j * NZ - j * (j - 1) / 2; }
};

// NZ consecutive values of a record (16-byte aligned records; an offset that is a
// multiple of NZ) with 16- or 8-byte loads and stores.
template <int NZ, typename T>
__device__ __forceinline__ void load_run(const T* p, T* out) {
  if constexpr (sizeof(T) == 4 && NZ % 4 == 0) {
#pragma unroll
    for (int k = 0; k < NZ; k += 4) {
      const float4 v = *reinterpret_cast<const float4*>(p + k);
      out[k] = v.x;
      out[k + 1] = v.y;
      out[k + 2] = v.z;
      out[k + 3] = v.w;
    }
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < NZ; k += 2) {
      const float2 v = *reinterpret_cast<const float2*>(p + k);
      out[k] = v.x;
      out[k + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NZ; k += 2) {
      const double2 v = *reinterpret_cast<const double2*>(p + k);
      out[k] = v.x;
      out[k + 1] = v.y;
    }
  }
}

template <int NZ, typename T>
__device__ __forceinline__ void store_run(const T* v, T* p) {
  if constexpr (sizeof(T) == 4 && NZ % 4 == 0) {
#pragma unroll
    for (int k = 0; k < NZ; k += 4)
      *reinterpret_cast<float4*>(p + k) = make_float4(v[k], v[k + 1], v[k + 2], v[k + 3]);
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < NZ; k += 2) *reinterpret_cast<float2*>(p + k) = make_float2(v[k], v[k + 1]);
  } else {
#pragma unroll
    for (int k = 0; k < NZ; k += 2) *reinterpret_cast<double2*>(p + k) = make_double2(v[k], v[k + 1]);
  }
}

template <typename T>
__device__ __forceinline__ T block_sum_all(T v, T* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T s = T(0);
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

template <typename T>
__device__ __forceinline__ void stage_spheres(const TrajArgs<T>& ta, const TrajCtx& cx, T* s_sph) {
  for (int i = threadIdx.x; i < 4 * cx.pr.M; i += blockDim.x) {
    const int m = i >> 2, c = i & 3;
    s_sph[i] = (T)ta.sph[cx.pr.sph + c * cx.pr.sph_ld + m];
  }
}

template <typename T>
__device__ __forceinline__ void load_pose(const TrajArgs<T>& ta, const TrajCtx& cx, int t, T* Tt) {
#pragma unroll
  for (int c = 0; c < 12; ++c) Tt[c] = (T)ta.task[cx.pr.task + c * cx.pr.task_ld + t];
}

// Bending coordinates of segment i of the start (end = 0) or goal (end = 1)
// configuration of a trajectory problem.
template <int NS, typename T, typename TR>
__device__ __forceinline__ void load_end(const TrajArgs<T>& ta, const TrajCtx& cx, int end, int i, TR r, TR* za,
                                         TR* zb) {
  const double* u = ta.task + cx.pr.task + (int64_t)(end * 3 * NS + 3 * i) * cx.pr.task_ld;
  u_to_ab((TR)u[0], (TR)u[cx.pr.task_ld], (TR)u[2 * cx.pr.task_ld], r, za, zb);
}

// Work list of the clearance term of one trajectory.  Every waypoint lane stores
// its segment base frames and pushes the (waypoint, segment, sphere) triples that
// pass the segment-ball test; then all lanes of the workgroup share the
// (triple, backbone point) pairs, so a few colliding waypoints do not hold the
// whole wave in their point loops.
template <typename T>
struct CollList {
  static constexpr int FR = 14;
  T* fr;      // [(t * NS + i) * FR]: rows 0 and 1 of the base rotation (6), base position (3), a, b,
              // arc midpoint (3); row 2 is their cross product
  static constexpr int OP = 6, OA = 9, OM = 11;
  int* list;  // packed triples (t << 12) | (i << 9) | m, one slice per wave
  int* cnt;   // entries per wave (at most 4 waves)
  int cap;    // 0: no list, each lane loops over its own points
};

// Base rotation of a frame record: rows 0 and 1 as stored, row 2 = row 0 x row 1
// (a rotation's rows form a right-handed orthonormal triple).
template <typename T>
__device__ __forceinline__ void frame_rot(const T* fr, T* R) {
#pragma unroll
  for (int k = 0; k < 6; ++k) R[k] = fr[k];
  R[6] = R[1] * R[5] - R[2] * R[4];
  R[7] = R[2] * R[3] - R[0] * R[5];
  R[8] = R[0] * R[4] - R[1] * R[3];
}

// The list area follows the other LDS arrays: frames, then the counter and the
// packed triples.
template <int NS, typename T>
__device__ __forceinline__ CollList<T> coll_list(T* area, int Tn, int cap) {
  CollList<T> cl;
  cl.fr = area;
  cl.cnt = reinterpret_cast<int*>(area + Tn * NS * CollList<T>::FR);
  cl.list = cl.cnt + 4;
  cl.cap = cap;
  return cl;
}

// Clearance residual of one backbone point x against sphere sm, squared / 2.
template <typename T>
__device__ __forceinline__ T point_sphere_cost(const T* x, const T* sm, T reach, T sqc) {
  const T d0 = x[0] - sm[0], d1 = x[1] - sm[1], d2 = x[2] - sm[2];
  const T q = d0 * d0 + d1 * d1 + d2 * d2;
  if (!(q < reach * reach)) return T(0);
  const T viol = reach - tsqrt(q);
  if (!(viol > T(0))) return T(0);
  const T rr = sqc * viol;
  return T(0.5) * rr * rr;
}

// Lane t (waypoints within the horizon): base frame and arc midpoint of every
// segment of waypoint t, into the list's frame area; the tip frame into Rt, pt.
template <int NS, typename T>
__device__ __forceinline__ void coll_frames(const RobotT<T>& rb, const T* z, int t, const CollList<T>& cl, T* Rt,
                                            T* pt) {
  T Rc[9], pc[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = (k % 4 == 0) ? T(1) : T(0);
  pc[0] = pc[1] = pc[2] = T(0);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const T a = z[2 * i], b = z[2 * i + 1], s = a * a + b * b;
    T* fr = cl.fr + (t * NS + i) * CollList<T>::FR;
#pragma unroll
    for (int k = 0; k < 6; ++k) fr[k] = Rc[k];
    fr[CollList<T>::OP] = pc[0];
    fr[CollList<T>::OP + 1] = pc[1];
    fr[CollList<T>::OP + 2] = pc[2];
    fr[CollList<T>::OA] = a;
    fr[CollList<T>::OA + 1] = b;
    seg_point(Rc, pc, a, b, rb.L[i], s, T(0.5), fr + CollList<T>::OM);
    ArcCoef<T> c = arc_coef<T, false>(s);
    T Ri[9], di[3], q[3], Rn[9];
    seg_R_d(a, b, rb.L[i], c, Ri, di);
    mv3(Rc, di, q);
    pc[0] += q[0];
    pc[1] += q[1];
    pc[2] += q[2];
    mm3(Rc, Ri, Rn);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = Rn[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) Rt[k] = Rc[k];
  pt[0] = pc[0];
  pt[1] = pc[1];
  pt[2] = pc[2];
}

template <int NS, typename T>
__device__ __forceinline__ void seg_consts(const RobotT<T>& rb, int i, T& Li, T& ri) {
  Li = rb.L[0];
  ri = rb.r[0];
#pragma unroll
  for (int q = 1; q < NS; ++q)
    if (q == i) {
      Li = rb.L[q];
      ri = rb.r[q];
    }
}

// All lanes, after the frames are stored: segment-ball tests with one sphere per
// lane (chunks of 64 spheres) against every (waypoint, segment).  Each wave owns a
// slice of the list and takes its pairs t * NS + i in a strided order; hits are
// placed with a ballot in (pair, sphere) order, so the list, and every sum over
// it, is the same on every run.  Hits that do not fit are evaluated by their
// lane; returns that cost.
template <int NS, typename T>
__device__ __forceinline__ T coll_enqueue(const RobotT<T>& rb, const WeightsT<T>& w, const T* s_sph, int M, int Tn,
                                          const CollList<T>& cl) {
  const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6), nwv = (int)((blockDim.x + 63) >> 6);
  const int capw = cl.cap / nwv;
  int* wl = cl.list + wv * capw;
  const int K = rb.K;
  const T invK = T(1) / T(K);
  const int npair = Tn * NS;
  int used = 0;  // entries of this wave so far (uniform across the wave)
  T cost = T(0);
  for (int m0 = 0; m0 < M; m0 += 64) {
    const int m = m0 + lane;
    const bool has = m < M;
    const T* sm = s_sph + 4 * (has ? m : 0);
    const T c0 = sm[0], c1 = sm[1], c2 = sm[2], rs = sm[3];
    // four (waypoint, segment) pairs per round: their midpoint loads are issued
    // together before the ballots serialise the placement
    for (int pr0 = wv; pr0 < npair; pr0 += 4 * nwv) {
      bool hit[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int pr = pr0 + j * nwv;
        const int prc = pr < npair ? pr : npair - 1;
        const int i = prc % NS;
        T Li, ri;
        seg_consts<NS>(rb, i, Li, ri);
        const T* fr = cl.fr + prc * CollList<T>::FR;
        const T* mid = fr + CollList<T>::OM;
        const T e0 = mid[0] - c0, e1 = mid[1] - c1, e2 = mid[2] - c2;
        const T rq = (rs + ri + w.margin + T(0.5) * Li) * T(1.0001);
        hit[j] = has && pr < npair && e0 * e0 + e1 * e1 + e2 * e2 < rq * rq;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned long long mask = __ballot(hit[j]);
        if (mask == 0ull) continue;
        const int pr = pr0 + j * nwv;
        const int t = pr / NS, i = pr - t * NS;
        const int rank =
            (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
        const int slot = used + rank;
        used += __popcll(mask);
        if (!hit[j]) continue;
        if (slot < capw) {
          wl[slot] = (t << 12) | (i << 9) | m;
        } else {
          T Li, ri;
          seg_consts<NS>(rb, i, Li, ri);
          const T* fr = cl.fr + pr * CollList<T>::FR;
          const T a = fr[CollList<T>::OA], b = fr[CollList<T>::OA + 1];
          T Rb[9];
          frame_rot(fr, Rb);
          for (int k = 1; k <= K; ++k) {
            T x[3];
            seg_point(Rb, fr + CollList<T>::OP, a, b, Li, a * a + b * b, T(k) * invK, x);
            cost += point_sphere_cost(x, sm, rs + ri + w.margin, w.sq_coll);
          }
        }
      }
    }
  }
  if (lane == 0) cl.cnt[wv] = used < capw ? used : capw;
  return cost;
}

// All lanes: every listed (waypoint, segment, sphere) triple, split into runs of
// at most 8 backbone points; a run whose own ball (around its middle arc point)
// misses the sphere is skipped.  Work items (triple, run) are strided over the
// workgroup.
template <int NS, typename T>
__device__ __forceinline__ T coll_drain(const RobotT<T>& rb, const WeightsT<T>& w, const T* s_sph,
                                        const CollList<T>& cl) {
  const int K = rb.K, nth = (int)blockDim.x, nwv = (nth + 63) >> 6;
  const int Q = (K + 7) >> 3;
  const int capw = cl.cap / nwv;
  const T invK = T(1) / T(K);
  const int de = nth / Q, dq = nth - de * Q;
  T cost = T(0);
  for (int wv = 0; wv < nwv; ++wv) {
    const int* wl = cl.list + wv * capw;
    const int total = cl.cnt[wv] * Q;
    int e = (int)threadIdx.x / Q, q = (int)threadIdx.x - e * Q;
    for (int wi = (int)threadIdx.x; wi < total; wi += nth) {
      const int code = wl[e];
      const int t = code >> 12, i = (code >> 9) & 7, m = code & 511;
      T Li, ri;
      seg_consts<NS>(rb, i, Li, ri);
      const T* fr = cl.fr + (t * NS + i) * CollList<T>::FR;
      const T a = fr[CollList<T>::OA], b = fr[CollList<T>::OA + 1], s = a * a + b * b;
      T Rb[9];
      frame_rot(fr, Rb);
      const T* pb = fr + CollList<T>::OP;
      const T* sm = s_sph + 4 * m;
      const T reach = sm[3] + ri + w.margin;
      const int k0 = 8 * q + 1, k1 = 8 * q + 8 < K ? 8 * q + 8 : K;
      T xc[3];
      seg_point(Rb, pb, a, b, Li, s, T(k0 + k1) * T(0.5) * invK, xc);
      const T d0 = xc[0] - sm[0], d1 = xc[1] - sm[1], d2 = xc[2] - sm[2];
      const T rq = (reach + T(k1 - k0) * T(0.5) * invK * Li) * T(1.0001);
      if (d0 * d0 + d1 * d1 + d2 * d2 < rq * rq) {
        for (int k = k0; k <= k1; ++k) {
          T x[3];
          seg_point(Rb, pb, a, b, Li, s, T(k) * invK, x);
          cost += point_sphere_cost(x, sm, reach, w.sq_coll);
        }
      }
      e += de;
      q += dq;
      if (q >= Q) {
        q -= Q;
        ++e;
      }
    }
  }
  return cost;
}

// Cost of one trajectory (value only), all lanes of the workgroup participate;
// lane t evaluates waypoint t.  If pen != NULL the collision part alone is also
// returned (every other weight zeroed).  s_u, s_p: LDS scratch of (H+1)*3n and
// (H+1)*3 values.
template <int NS, typename T>
__device__ __forceinline__ T traj_cost(const RobotT<T>& rb, const WeightsT<T>& w, const TrajArgs<T>& ta,
                                       const TrajCtx& cx, const T* z, const T* s_sph, T* s_u, T* s_p, T* s_red, T* pen,
                                       const CollList<T>& cl) {
  constexpr int NU = 3 * NS;
  const int t = threadIdx.x, H = cx.pr.Tn - 1, M = cx.pr.M;
  const bool act = t <= H;
  const bool listed = cl.cap > 0 && M > 0;
  T cst = T(0), cpen = T(0);
  T Rt[9], pt[3];  // tip frame of waypoint t
  if (listed) {
    if (act) coll_frames<NS>(rb, z, t, cl, Rt, pt);
    __syncthreads();
    cpen = coll_enqueue<NS>(rb, w, s_sph, M, H + 1, cl);
    cst = cpen;
  }
  if (act) {
    // bound hinges in the working precision, as in the normal equations
    if (listed) {
      cst += bounds_cost<NS>(rb, w, z);
    } else if (M == 0) {
      fk_tip<NS>(rb, z, Rt, pt);
      cst = bounds_cost<NS>(rb, w, z);
    } else {
      Fwd<NS, T> f;
      WeightsT<T> wb = w;  // clearance alone here; the bounds below
      wb.sq_lim = wb.sq_curv = T(0);
      cpen = config_forward<NS, T, false>(rb, wb, z, s_sph, M, 4, 1, f);
      cst = cpen + bounds_cost<NS>(rb, w, z);
#pragma unroll
      for (int k = 0; k < 9; ++k) Rt[k] = f.R[k];
      pt[0] = f.p[0];
      pt[1] = f.p[1];
      pt[2] = f.p[2];
    }
    if (ta.kind == CR_KIND_PATH) {
      T Tt[12], ft[3], tq[3];
      load_pose(ta, cx, t, Tt);
      cst += pose_term<T, false>(w, Rt, pt, Tt, ft, tq);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      T u[3];
      ab_to_u(z[2 * i], z[2 * i + 1], rb.r[i], u);
#pragma unroll
      for (int j = 0; j < 3; ++j) s_u[t * NU + 3 * i + j] = u[j];
    }
    s_p[3 * t] = pt[0];
    s_p[3 * t + 1] = pt[1];
    s_p[3 * t + 2] = pt[2];
  }
  __syncthreads();
  if (listed) {
    const T part = coll_drain<NS>(rb, w, s_sph, cl);
    cst += part;
    cpen += part;
  }
  if (act) {
    const T idt = T(1) / w.dt, idt2 = idt * idt;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      if (t >= 1) {
        const T v = (s_u[t * NU + m] - s_u[(t - 1) * NU + m]) * idt;
        const T rr = w.sq_vel * v;
        cst += T(0.5) * rr * rr;
        if (w.has_vmax && fabs(v) > w.v_max) {
          const T hr = w.sq_lim * (fabs(v) - w.v_max);
          cst += T(0.5) * hr * hr;
        }
      }
      if (t >= 2) {
        const T a = (s_u[t * NU + m] - T(2) * s_u[(t - 1) * NU + m] + s_u[(t - 2) * NU + m]) * idt2;
        const T rr = w.sq_acc * a;
        cst += T(0.5) * rr * rr;
        if (w.has_amax && fabs(a) > w.a_max) {
          const T hr = w.sq_lim * (fabs(a) - w.a_max);
          cst += T(0.5) * hr * hr;
        }
      }
    }
    if (ta.kind == CR_KIND_TRAJ) {
      if (t >= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T rr = w.sq_len * (s_p[3 * t + c] - s_p[3 * (t - 1) + c]);
          cst += T(0.5) * rr * rr;
        }
      }
      if (t == 0 || t == H) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          T za, zb;
          load_end<NS>(ta, cx, t == 0 ? 0 : 1, i, rb.r[i], &za, &zb);
          const T ra = w.sq_eq * (z[2 * i] - za), rb2 = w.sq_eq * (z[2 * i + 1] - zb);
          cst += T(0.5) * (ra * ra + rb2 * rb2);
        }
      }
    }
  }
  const T total = block_sum_all(cst, s_red);
  if (pen) *pen = block_sum_all(cpen, s_red);
  return total;
}

// ---------------------------------------------------------------------------

// Exploration stage of path following (Sec. IV-B): IK at every (seed, waypoint)
// of stage 1 against that waypoint's reference pose, the plain method for
// `iters` iterations (with the problem's spheres).  One workgroup per
// trajectory, one lane per waypoint.  cand has the layout of Z; okf: 2 = passes
// the success test, 1 = finite, 0 = not finite.
template <int NS, typename T>
__global__ void __launch_bounds__(64)
    k_path_wp_ik(RobotT<T> rb, WeightsT<T> w, LMOpts<T> o, TrajArgs<T> ta, const double* __restrict__ useed,
                 int iters, T lam0, T* __restrict__ cand, int32_t* __restrict__ okf) {
  constexpr int NZ = 2 * NS;
  const TrajCtx cx = traj_ctx(ta, blockIdx.x);
  const int M = cx.pr.M;
  const double* sp = M > 0 ? ta.sph + cx.pr.sph : nullptr;
  for (int t = threadIdx.x; t < cx.pr.Tn; t += blockDim.x) {
    T tt[12];
    load_pose(ta, cx, t, tt);
    const double* u = useed + cx.pr.seed + (int64_t)cx.s * cx.pr.Tn + t;
    T z[NZ];
#pragma unroll
    for (int i = 0; i < NS; ++i)
      u_to_ab((T)u[(3 * i) * cx.pr.seed_ld], (T)u[(3 * i + 1) * cx.pr.seed_ld], (T)u[(3 * i + 2) * cx.pr.seed_ld],
              rb.r[i], &z[2 * i], &z[2 * i + 1]);
    T lam = lam0;
    bool failed = false;
    int trials = 0;
    if (M > 0) lm_cfg<NS, T, double>(rb, w, tt, z, lam, iters, o, failed, trials, sp, M, 1, cx.pr.sph_ld);
    else lm_ik<NS>(rb, w, tt, z, lam, iters, o, failed, trials);
    bool fin = !failed;
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
      fin = fin && tfinite(z[k]);
      cand[(cx.wp + t) * NZ + k] = z[k];
    }
    okf[cx.wp + t] = !fin ? 0 : (ik_success<NS, T>(rb, z, tt, sp, M, cx.pr.sph_ld) ? 2 : 1);
  }
}

// Path assembly: path s starts at seed s's waypoint-0 solution; every later
// waypoint takes, among the problem's S solutions there that pass the success
// test, the nearest to the path's previous waypoint in the infinity norm over z
// (ties: lower seed); if none passes, the nearest finite one; if none is finite,
// the previous waypoint again.  One lane per trajectory.
template <int NS, typename T>
__global__ void __launch_bounds__(256)
    k_path_chain(TrajArgs<T> ta, int64_t nt, const T* __restrict__ cand, const int32_t* __restrict__ okf,
                 T* __restrict__ Z) {
  constexpr int NZ = 2 * NS;
  const int64_t traj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (traj >= nt) return;
  const TrajCtx cx = traj_ctx(ta, traj);
  const int Tn = cx.pr.Tn, S = cx.pr.S;
  T prev[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    prev[k] = cand[cx.wp * NZ + k];
    Z[cx.wp * NZ + k] = prev[k];
  }
  for (int t = 1; t < Tn; ++t) {
    int best = -1;
    T bd = T(0);
    for (int pass = 0; pass < 2 && best < 0; ++pass) {
      for (int j = 0; j < S; ++j) {
        const int64_t at = cx.pr.wp0 + (int64_t)j * Tn + t;
        const int f = okf[at];
        if (pass == 0 ? f != 2 : f < 1) continue;
        T d = T(0);
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
          const T e = fabs(cand[at * NZ + k] - prev[k]);
          d = e > d ? e : d;
        }
        if (best < 0 || d < bd) {
          best = j;
          bd = d;
        }
      }
    }
    if (best >= 0) {
      const int64_t at = cx.pr.wp0 + (int64_t)best * Tn + t;
#pragma unroll
      for (int k = 0; k < NZ; ++k) prev[k] = cand[at * NZ + k];
    }
#pragma unroll
    for (int k = 0; k < NZ; ++k) Z[(cx.wp + t) * NZ + k] = prev[k];
  }
}

// Stage-1 state from the seeds: one workgroup per trajectory, lane t = waypoint.
template <int NS, typename T>
__global__ void __launch_bounds__(256)
    k_traj_init(RobotT<double> rbd, TrajArgs<T> ta, const double* __restrict__ useed, T* __restrict__ Z) {
  const TrajCtx cx = traj_ctx(ta, blockIdx.x);
  for (int t = threadIdx.x; t < cx.pr.Tn; t += blockDim.x) {
    const double* u = useed + cx.pr.seed + (int64_t)cx.s * cx.pr.Tn + t;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      double a, b;
      u_to_ab(u[(3 * i) * cx.pr.seed_ld], u[(3 * i + 1) * cx.pr.seed_ld], u[(3 * i + 2) * cx.pr.seed_ld], rbd.rd[i], &a,
              &b);
      Z[(cx.wp + t) * 2 * NS + 2 * i] = (T)a;
      Z[(cx.wp + t) * 2 * NS + 2 * i + 1] = (T)b;
    }
  }
}

// OCC: the minimum waves per SIMD the register allocation must allow (1 = the
// compiler's own choice); the autotuner picks among the compiled targets.
template <int NS, typename T, int OCC = 1, int G = 1>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC)))
    k_traj_build(RobotT<T> rb, WeightsT<T> w, TrajArgs<T> ta, const T* __restrict__ Z, T* __restrict__ blk,
                 T* __restrict__ cost0, int32_t* __restrict__ failed, int64_t nt, int lds_per) {
  constexpr int NZ = 2 * NS, NU = 3 * NS, NP = NZ * (NZ + 1) / 2;
  using R = Rec<NS>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // G trajectories per workgroup (2 for horizons of at most 32 waypoints: one per
  // half-wave), each with its own lds_per values of LDS
  const int Tp = G == 1 ? (int)blockDim.x : 32;
  const int sub = G == 1 ? 0 : (int)threadIdx.x / Tp;
  const int t = (int)threadIdx.x - sub * Tp;
  const int64_t traj = (int64_t)blockIdx.x * G + sub;
  const bool live = traj < nt && !failed[traj];
  if (G == 1 && !live) return;  // uniform per workgroup
  TrajCtx cx;
  cx.pr.Tn = 0;
  cx.pr.M = 0;
  cx.wp = 0;
  if (live) cx = traj_ctx(ta, traj);
  const int Tn = cx.pr.Tn, H = Tn - 1, M = cx.pr.M;
  T* s_sph = reinterpret_cast<T*>(smem_raw) + (size_t)sub * lds_per;
  T* s_u = s_sph + 4 * M;
  T* s_p = s_u + Tn * NU;
  T* s_jp = s_p + Tn * 3;
  T* s_red = s_jp + Tn * 3 * NZ;
  for (int i = t; i < 4 * M; i += Tp) {
    const int m = i >> 2, c = i & 3;
    s_sph[i] = (T)ta.sph[cx.pr.sph + c * cx.pr.sph_ld + m];
  }
  __syncthreads();
  const bool act = live && t < Tn;
  T z[NZ], Hp[NP], g[NZ], ptip[3], Jp[3][NZ];
  T cst = T(0);
  if (act) {
#pragma unroll
    for (int k = 0; k < NZ; ++k) z[k] = Z[(cx.wp + t) * NZ + k];
    T Tt[12];
    if (ta.kind == CR_KIND_PATH) {
      load_pose(ta, cx, t, Tt);
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) Tt[k] = T(0);
    }
    cst = local_normal_eq<NS, T, T>(rb, w, z, s_sph, M, 4, 1, Tt, Hp, g, ptip, Jp, ta.kind == CR_KIND_PATH);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      T u[3];
      ab_to_u(z[2 * i], z[2 * i + 1], rb.r[i], u);
#pragma unroll
      for (int j = 0; j < 3; ++j) s_u[t * NU + 3 * i + j] = u[j];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s_p[3 * t + c] = ptip[c];
#pragma unroll
      for (int k = 0; k < NZ; ++k) s_jp[(t * 3 + c) * NZ + k] = Jp[c][k];
    }
  }
  __syncthreads();
  if (act) {
    // The smoothness couplings of H_{t,t-1} and H_{t,t-2} act on each segment's
    // own lifts, so they are 2x2 symmetric blocks on the diagonal: (aa, ab, bb)
    // per segment.  The path-length coupling is added when the record is written.
    T Bs[NS][3], Cs[NS][3];
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) Bs[i][k] = Cs[i][k] = T(0);
    const T idt = T(1) / w.dt, idt2 = idt * idt;
    // tendon velocity / acceleration smoothness and their hinges (linear in the lifts)
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int ca = 2 * i, cb = 2 * i + 1;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int m = 3 * i + j;
        T ja, jb;
        lift_row(j, rb.r[i], &ja, &jb);
        const T o00 = ja * ja, o01 = ja * jb, o11 = jb * jb;
        auto add_self = [&](T c1, T rr) {  // row with coefficient c1 on u_t
          g[ca] += c1 * rr * ja;
          g[cb] += c1 * rr * jb;
          Hp[tri(ca, ca)] += c1 * c1 * o00;
          Hp[tri(cb, ca)] += c1 * c1 * o01;
          Hp[tri(cb, cb)] += c1 * c1 * o11;
        };
        auto add_off = [&](T* X, T c1c2) {  // coupling block entry c1 c2 lift^T lift
          X[0] += c1c2 * o00;
          X[1] += c1c2 * o01;
          X[2] += c1c2 * o11;
        };
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int tau = t + k;
          if (tau >= 1 && tau <= H) {
            const T v = (s_u[tau * NU + m] - s_u[(tau - 1) * NU + m]) * idt;
            const T rr = w.sq_vel * v;
            const T cs = (k == 0 ? idt : -idt) * w.sq_vel;
            if (k == 0) cst += T(0.5) * rr * rr;
            add_self(cs, rr);
            if (k == 0) add_off(Bs[i], cs * (-idt * w.sq_vel));
            if (w.has_vmax && fabs(v) > w.v_max) {
              const T sg = v < T(0) ? -w.sq_lim : w.sq_lim;
              const T hr = w.sq_lim * (fabs(v) - w.v_max);
              const T hs = sg * (k == 0 ? idt : -idt);
              if (k == 0) cst += T(0.5) * hr * hr;
              add_self(hs, hr);
              if (k == 0) add_off(Bs[i], hs * (sg * -idt));
            }
          }
        }
        const T cf[3] = {T(1), T(-2), T(1)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int tau = t + k;
          if (tau >= 2 && tau <= H) {
            const T a = (s_u[tau * NU + m] - T(2) * s_u[(tau - 1) * NU + m] + s_u[(tau - 2) * NU + m]) * idt2;
            const T rr = w.sq_acc * a;
            const T cs = cf[k] * idt2 * w.sq_acc;
            if (k == 0) cst += T(0.5) * rr * rr;
            add_self(cs, rr);
            if (k <= 1) add_off(Bs[i], cs * cf[k + 1] * idt2 * w.sq_acc);
            if (k == 0) add_off(Cs[i], cs * cf[2] * idt2 * w.sq_acc);
            if (w.has_amax && fabs(a) > w.a_max) {
              const T sg = a < T(0) ? -w.sq_lim : w.sq_lim;
              const T hr = w.sq_lim * (fabs(a) - w.a_max);
              const T hs = sg * cf[k] * idt2;
              if (k == 0) cst += T(0.5) * hr * hr;
              add_self(hs, hr);
              if (k <= 1) add_off(Bs[i], hs * sg * cf[k + 1] * idt2);
              if (k == 0) add_off(Cs[i], hs * sg * cf[2] * idt2);
            }
          }
        }
      }
    }
    if (ta.kind == CR_KIND_TRAJ) {
      // tip path length, eq. (11) squared, couples t and t - 1
      const T sl2 = w.sq_len * w.sq_len;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T sw = T(0);  // multiplicity of J_p^T J_p on the diagonal block
        T gr = T(0);
        if (t >= 1) {
          const T rr = w.sq_len * (s_p[3 * t + c] - s_p[3 * (t - 1) + c]);
          cst += T(0.5) * rr * rr;
          gr += w.sq_len * rr;
          sw += sl2;
        }
        if (t + 1 <= H) {
          const T rr = w.sq_len * (s_p[3 * (t + 1) + c] - s_p[3 * t + c]);
          gr -= w.sq_len * rr;
          sw += sl2;
        }
#pragma unroll
        for (int a = 0; a < NZ; ++a) {
          g[a] += gr * Jp[c][a];
#pragma unroll
          for (int b = 0; b <= a; ++b) Hp[tri(a, b)] += sw * Jp[c][a] * Jp[c][b];
        }
      }
      // endpoint equalities, penalised (eq. 17)
      if (t == 0 || t == H) {
        const T se2 = w.sq_eq * w.sq_eq;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          T za, zb;
          load_end<NS>(ta, cx, t == 0 ? 0 : 1, i, rb.r[i], &za, &zb);
          const T ra = w.sq_eq * (z[2 * i] - za), rb2 = w.sq_eq * (z[2 * i + 1] - zb);
          cst += T(0.5) * (ra * ra + rb2 * rb2);
          g[2 * i] += w.sq_eq * ra;
          g[2 * i + 1] += w.sq_eq * rb2;
          Hp[tri(2 * i, 2 * i)] += se2;
          Hp[tri(2 * i + 1, 2 * i + 1)] += se2;
        }
      }
    }
    T* rec = blk + (cx.wp + t) * R::SIZE;
#pragma unroll
    for (int k = 0; k < NP; ++k) rec[R::OHI + k] = Hp[k];  // lower triangle, packed by rows
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        rec[R::OBS + 3 * i + k] = Bs[i][k];
        rec[R::OCS + 3 * i + k] = Cs[i][k];
      }
    if (ta.kind == CR_KIND_TRAJ) {
      // H_{t,t-1} in full: the smoothness blocks minus the path-length coupling
      // sq_len^2 J_p(t)^T J_p(t-1)
      const bool len = t >= 1;
      const T sl2 = w.sq_len * w.sq_len;
      T jq[3][NZ] = {};  // J_p at t - 1
      if (len) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int b = 0; b < NZ; ++b) jq[q][b] = s_jp[((t - 1) * 3 + q) * NZ + b];
      }
#pragma unroll
      for (int a = 0; a < NZ; ++a) {
        T brow[NZ];  // row a of H_{t,t-1}
#pragma unroll
        for (int b = 0; b < NZ; ++b) {
          T bv = a / 2 == b / 2 ? Bs[a / 2][(a & 1) + (b & 1)] : T(0);
          if (len) bv -= sl2 * (Jp[0][a] * jq[0][b] + Jp[1][a] * jq[1][b] + Jp[2][a] * jq[2][b]);
          brow[b] = bv;
        }
        store_run<NZ>(brow, rec + R::OB + a * NZ);
      }
    }
#pragma unroll
    for (int k = 0; k < NZ; ++k) rec[R::OG + k] = g[k];
  }
  T total;
  if constexpr (G == 1) {
    total = block_sum_all(cst, s_red);
  } else {  // the trajectory's half-wave
    total = cst;
    for (int off = Tp >> 1; off > 0; off >>= 1) total += __shfl_xor(total, off, Tp);
  }
  if (live && t == 0) {
    cost0[traj] = total;
    if (!tfinite(total)) failed[traj] = 1;
  }
}

// Block Cholesky of the block-pentadiagonal H + lambda D, in place, then
// y = L^-1 (-g), delta = L^-T y and g.delta, from both ends of the trajectory at
// once.  2 NZ lanes own one trajectory: the top group (row a on lane a) factors
// waypoints 0 .. m-1 forward, the bottom group factors waypoints Tn-1 .. m+2 in
// reverse order (the same recurrences on the reversed matrix, whose couplings are
// the transposed blocks), then eliminates its part from the two middle waypoints
// m, m+1 (their Schur complement), and the top group factors those two last.  The
// backward substitution starts at the middle and runs outward on both groups.
// For Tn < 4 the top group does everything.  The sequential chain is thus about
// Tn / 2 + 4 steps instead of Tn, on twice the lanes.
// Storage of the factor (records of the workspace): the top group stores row a of
// L_tt and L_{t,t-1} in record t (OL, OB); the bottom group, whose chain
// predecessors of waypoint r are r+1 and r+2, stores row a of its coupling block
// to r+1 in record r+1 (OB), so that each of its backward steps finds that
// coupling in its own record and no input is overwritten before it is read.  The
// couplings two apart are formed again from the segment blocks in the backward
// pass.  The last factors, y and delta of each group are
// in LDS (diagonal factors packed by rows); the middle downdates go from the
// bottom group to the top group through the bottom group's free LDS slots.
// Rows are exchanged only within a wave (workgroup = one wave).  In FP32 the
// diagonal block is exchanged once and factored redundantly by each row lane; in
// FP64 it is factored by rounds over its columns (one LDS exchange per column).
template <int NS, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (NS <= 4 ? 4 : (NS == 5 ? 3 : 1)) : 1)))
    k_traj_solve(TrajArgs<T> ta, int64_t nt, T* __restrict__ blk, const T* __restrict__ lam, const int32_t* __restrict__ failed,
                 int32_t* __restrict__ chol_ok, T* __restrict__ gd_out) {
  constexpr int NZ = 2 * NS, G2 = 64 / (2 * NZ), NG = 2 * G2, NP = NZ * (NZ + 1) / 2;
  constexpr int RS = NZ + (NZ & 1);  // LDS row stride
  constexpr int GS = NZ * RS + 4;    // LDS stride of a full block (breaks bank aliasing between groups)
  constexpr int PS = NP + 4;         // LDS stride of a packed triangle
  using R = Rec<NS>;
  __shared__ T sL[3][NG * PS];     // L_pp of chain positions p mod 3, packed by rows
  __shared__ T sD[3][NG * RS];     // 1 / diag(L_pp)
  __shared__ T sB[NG * GS];        // coupling of the last position to the one before it
  __shared__ T sX[NG * GS];        // rows of the coupling being formed (for the symmetric updates)
  __shared__ T sY[3][NG * RS];     // y_p, later delta, of positions p mod 3
  const int lane = threadIdx.x;
  const bool inw = lane < NG * NZ;  // lane owns a row
  const int gg = inw ? lane / NZ : 0, a = inw ? lane - gg * NZ : 0, base = gg * NZ;
  const int half = gg & 1, j2 = gg >> 1, pg = gg ^ 1;  // 0: top, 1: bottom; partner group
  const int64_t traj = (int64_t)blockIdx.x * G2 + j2;
  const bool act = inw && traj < nt && !failed[traj];
  int Tn = 0;
  int64_t wp = 0;
  if (act) {
    const TrajCtx cx = traj_ctx(ta, traj);
    Tn = cx.pr.Tn;
    wp = cx.wp;
  }
  // chain geometry: the bottom group factors nbot waypoints, the top group m
  // before the middle pair (nbot = 0: the top group alone, all Tn)
  const int nbot = Tn >= 4 ? (Tn - 1) / 2 : 0;
  const int m = Tn >= 4 ? (Tn - 2) / 2 : Tn;
  const int ntop = Tn - nbot;
  const int nfull = half ? nbot : m;  // full steps of this group in the first phase
  const int Tm = ta.Tmax;
  const int K1 = Tm >= 4 ? max((Tm - 1) / 2, min(Tm, 3)) : Tm;  // first-phase steps of the launch
  const T lm = act ? lam[traj] : T(0);
  T* const recs = blk + wp * R::SIZE;
  bool ok = true;
  const bool dense_b = ta.kind == CR_KIND_TRAJ;
  const int sa = 3 * (a >> 1) + (a & 1);  // row a of the segment's (aa, ab, bb)
  // Inputs of the step at waypoint r: row a of H_rr (lower part), of the coupling
  // to the chain predecessor (top: H_{r,r-1} from record r; bottom: H_{r,r+1} =
  // H_{r+1,r}^T, column a of record r+1's block, or its symmetric segment blocks),
  // of the coupling two back (the segment blocks of record r or r+2, symmetric),
  // and g_a.  hb, hc: the couplings exist.
  auto load_step = [&](int r, bool hb, bool hc, T* h, T* bw, T* c, T& gv) {
    const T* rr = recs + (int64_t)r * R::SIZE;
#pragma unroll
    for (int b = 0; b < NZ; ++b) h[b] = b <= a ? rr[R::OHI + a * (a + 1) / 2 + b] : T(0);
    gv = rr[R::OG + a];
    const T* rb = half ? rr + R::SIZE : rr;
    const T* rc = half ? rr + 2 * R::SIZE : rr;
    if (hb) {
      if (dense_b) {
        if (half) {
#pragma unroll
          for (int b = 0; b < NZ; ++b) bw[b] = rb[R::OB + b * NZ + a];
        } else {
          load_run<NZ>(rb + R::OB + a * NZ, bw);
        }
      } else {
        const T b0 = rb[R::OBS + sa], b1 = rb[R::OBS + sa + 1];
#pragma unroll
        for (int b = 0; b < NZ; ++b) bw[b] = b == (a & ~1) ? b0 : (b == (a | 1) ? b1 : T(0));
      }
    } else {
#pragma unroll
      for (int b = 0; b < NZ; ++b) bw[b] = T(0);
    }
    if (hc) {
      const T c0 = rc[R::OCS + sa], c1 = rc[R::OCS + sa + 1];
#pragma unroll
      for (int b = 0; b < NZ; ++b) c[b] = b == (a & ~1) ? c0 : (b == (a | 1) ? c1 : T(0));
    } else {
#pragma unroll
      for (int b = 0; b < NZ; ++b) c[b] = T(0);
    }
  };
  auto row_of = [&](int p) { return half ? Tn - 1 - p : p; };
  // One step of the chain at position p (waypoint r), workgroup-uniform barriers.
  //   on: this lane's group works; hp1, hp2: the predecessors' factors exist;
  //   cross: the p - 1 coupling in sB is used even without hp1 (the middle);
  //   fac: factor the diagonal block (else S and y stay the downdates);
  //   S, y, Bw, Cc: row a of the damped diagonal block, y, the couplings;
  //   oB: where row a of the coupling to p - 1 goes (nullptr: nowhere);
  //   orec: record of the factor and y (nullptr: not stored).
  auto step = [&](bool on, int p, bool hp1, bool hp2, bool cross, bool fac, T* S, T& y, T* Bw, const T* Cc, T* oB,
                  T* orec) {
    const int s0 = p % 3, s1 = (p + 2) % 3, s2 = (p + 1) % 3;  // slots of p, p-1, p-2
    {
      // row a of L_{p,p-2} = H_{p,p-2} L_{p-2}^-T (forward substitution)
      const T* L2 = &sL[s2][gg * PS];
      const T* D2 = &sD[s2][gg * RS];
      T x[NZ];
#pragma unroll
      for (int i = 0; i < NZ; ++i) x[i] = on && hp2 ? Cc[i] : T(0);
      if (on && hp2) {
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
          T v = x[i];
#pragma unroll
          for (int j = 0; j < i; ++j) v -= L2[tri(i, j)] * x[j];
          x[i] = v * D2[i];
        }
        const T* Y2 = &sY[s2][gg * RS];
#pragma unroll
        for (int i = 0; i < NZ; ++i) y -= x[i] * Y2[i];
        if (hp1 || cross) {
          // H_{p,p-1} -= L_{p,p-2} L_{p-1,p-2}^T
          const T* B1 = &sB[gg * GS];
#pragma unroll
          for (int b = 0; b < NZ; ++b) {
            T v = T(0);
#pragma unroll
            for (int i = 0; i < NZ; ++i) v += x[i] * B1[b * RS + i];
            Bw[b] -= v;
          }
        }
      }
      __syncthreads();  // sB read
      if (inw) {
#pragma unroll
        for (int i = 0; i < NZ; ++i) sX[gg * GS + a * RS + i] = x[i];
      }
      __syncthreads();
      // S -= L_{p,p-2} L_{p,p-2}^T (row a)
      if (on && hp2) {
#pragma unroll
        for (int b = 0; b < NZ; ++b) {
          T v = T(0);
#pragma unroll
          for (int i = 0; i < NZ; ++i) v += x[i] * sX[gg * GS + b * RS + i];
          S[b] -= v;
        }
      }
      __syncthreads();
    }
    {
      // row a of L_{p,p-1} = (H_{p,p-1} - ...) L_{p-1}^-T
      const T* L1 = &sL[s1][gg * PS];
      const T* D1 = &sD[s1][gg * RS];
      T x[NZ];
#pragma unroll
      for (int i = 0; i < NZ; ++i) x[i] = T(0);
      if (on && hp1) {
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
          T v = Bw[i];
#pragma unroll
          for (int j = 0; j < i; ++j) v -= L1[tri(i, j)] * x[j];
          x[i] = v * D1[i];
        }
        const T* Y1 = &sY[s1][gg * RS];
#pragma unroll
        for (int i = 0; i < NZ; ++i) y -= x[i] * Y1[i];
        if (oB) store_run<NZ>(x, oB);
      }
      if (inw) {
#pragma unroll
        for (int i = 0; i < NZ; ++i) sX[gg * GS + a * RS + i] = x[i];
        // the coupling of this position to the previous one, for the next step
        // (the middle keeps its cross downdate there instead)
        if (on && (hp1 || !cross)) {
#pragma unroll
          for (int i = 0; i < NZ; ++i) sB[gg * GS + a * RS + i] = x[i];
        }
        if (on && cross) {
#pragma unroll
          for (int i = 0; i < NZ; ++i) sB[gg * GS + a * RS + i] = Bw[i];
        }
      }
      __syncthreads();
      if (on && hp1) {
#pragma unroll
        for (int b = 0; b < NZ; ++b) {
          T v = T(0);
#pragma unroll
          for (int i = 0; i < NZ; ++i) v += x[i] * sX[gg * GS + b * RS + i];
          S[b] -= v;
        }
      }
    }
    T* Lt = &sL[s0][gg * PS];
    T* Dt = &sD[s0][gg * RS];
    T* Yt = &sY[s0][gg * RS];
    if (!fac) {
      // the middle's downdates, packed like a factor, for the top group
      __syncthreads();
      if (inw && on) {
#pragma unroll
        for (int b = 0; b < NZ; ++b)
          if (b <= a) Lt[tri(a, b)] = S[b];
        Yt[a] = y;
      }
      __syncthreads();
      return;
    }
    if constexpr (sizeof(T) == 4) {
      // L L^T = S and y_p = L^-1 y in one exchange: the rows of S and y go to LDS
      // (the slot of position p - 3, no longer read), every lane of the group
      // factors the whole block in registers with the same arithmetic, and the
      // first lane publishes the factor for the rows and later positions.
      if (inw && on) {
#pragma unroll
        for (int b = 0; b < NZ; ++b)
          if (b <= a) Lt[tri(a, b)] = S[b];
        Yt[a] = y;
      }
      __syncthreads();
      T L[NP], yv[NZ], dv[NZ];
#pragma unroll
      for (int i = 0; i < NP; ++i) L[i] = Lt[i];
#pragma unroll
      for (int i = 0; i < NZ; ++i) yv[i] = Yt[i];
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        T dd = L[tri(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) dd -= L[tri(j, k)] * L[tri(j, k)];
        ok = ok && (!on || dd > T(0));
        // hardware square root and reciprocal (1 ulp each; dd > 0 is normal here or
        // replaced by 1), then products: the IEEE-exact forms cost about ten
        // instructions each and this block is factored on every row lane
        const T ljj = __builtin_amdgcn_sqrtf(dd > T(0) ? dd : T(1));
        L[tri(j, j)] = ljj;
        dv[j] = __builtin_amdgcn_rcpf(ljj);
        yv[j] = yv[j] * dv[j];
#pragma unroll
        for (int i = j + 1; i < NZ; ++i) {
          T v = L[tri(i, j)];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= L[tri(i, k)] * L[tri(j, k)];
          L[tri(i, j)] = v * dv[j];
          yv[i] -= L[tri(i, j)] * yv[j];
        }
      }
      __syncthreads();
      if (inw && on && a == 0) {
#pragma unroll
        for (int i = 0; i < NP; ++i) Lt[i] = L[i];
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
          Dt[i] = dv[i];
          Yt[i] = yv[i];
        }
      }
      __syncthreads();
      y = Yt[a];
      if (on && orec) {
        // column a of L_pp, rows a .. NZ - 1
#pragma unroll
        for (int k = 0; k < NZ; ++k)
          if (k >= a) orec[R::OL + R::lcol(a) + k - a] = Lt[tri(k, a)];
        orec[R::OY + a] = y;
      }
    } else {
      // L L^T = S and y_p = L^-1 y, column by column: in round j lane j finishes
      // its pivot and y_j and publishes its row; rows below take column j.
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        if (a == j) {
          T dd = S[j];
#pragma unroll
          for (int k = 0; k < j; ++k) dd -= S[k] * S[k];
          ok = ok && (!on || dd > T(0));
          const T ljj = tsqrt(dd > T(0) ? dd : T(1));
          S[j] = ljj;
          y = y / ljj;
          if (inw && on) {
#pragma unroll
            for (int k = 0; k <= j; ++k) Lt[tri(j, k)] = S[k];
            Dt[j] = T(1) / ljj;
            Yt[j] = y;
          }
        }
        __syncthreads();
        if (a > j) {
          T v = S[j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= S[k] * Lt[tri(j, k)];
          S[j] = v * Dt[j];
          y -= S[j] * Yt[j];
        }
      }
      if (on && orec) {
#pragma unroll
        for (int b = 0; b < NZ; ++b)
          if (b <= a) orec[R::OL + R::lcol(b) + a - b] = S[b];  // row a of L_pp
        orec[R::OY + a] = y;
      }
    }
    __syncthreads();
  };
  // damped diagonal row: H + lambda max(diag, 1e-12) on the pivot
  auto damp = [&](T* S) {
#pragma unroll
    for (int b = 0; b < NZ; ++b)
      if (b == a) S[b] += lm * (S[b] > T(1e-12) ? S[b] : T(1e-12));
  };
  // FP32 inputs of the next step are loaded while the current one is factored
  // (the chain is latency-bound)
  constexpr bool PF = sizeof(T) == 4 && NZ <= 10;
  T pH[NZ], pB[NZ], pC[NZ], pG = T(0);
  if constexpr (PF) {
    if (act && 0 < nfull) load_step(row_of(0), false, false, pH, pB, pC, pG);
  }
  // phase 1: full steps of both groups, positions 0 .. K1 - 1
  for (int p = 0; p < K1; ++p) {
    const bool on = act && p < nfull;
    const int r = row_of(p);
    T S[NZ], Bw[NZ], Cc[NZ], gv = T(0);
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < NZ; ++k) {
        S[k] = pH[k];
        Bw[k] = pB[k];
        Cc[k] = pC[k];
      }
      gv = pG;
      if (act && p + 1 < nfull) load_step(row_of(p + 1), p + 1 >= 1, p + 1 >= 2, pH, pB, pC, pG);
    } else {
      if (on) load_step(r, p >= 1, p >= 2, S, Bw, Cc, gv);
    }
    if (!on) {
#pragma unroll
      for (int b = 0; b < NZ; ++b) S[b] = T(b == a);
    } else {
      damp(S);
    }
    T y = on ? -gv : T(0);
    T* rec = recs + (int64_t)r * R::SIZE;
    T* oB = on && p >= 1 ? (half ? rec + R::SIZE : rec) + R::OB + a * NZ : nullptr;
    step(on, p, p >= 1, p >= 2, false, true, S, y, Bw, Cc, oB, on ? rec : nullptr);
  }
  // phase 2: the bottom group's part of the middle's Schur complement: waypoint
  // m + 1 (predecessors m + 2, m + 3), then m (predecessor m + 2 two back; the
  // cross term with m + 1 is left in sB); results packed in the slots of
  // positions nbot and nbot + 1
  const bool mid = act && nbot > 0;
  for (int q = 0; q < 2; ++q) {
    const bool on = mid && half;
    const int p = nbot + q, r = m + 1 - q;
    T S[NZ], Bw[NZ], Cc[NZ], gv;
#pragma unroll
    for (int b = 0; b < NZ; ++b) S[b] = T(0);
    if (on) {
      // couplings of waypoint m + 1 to m + 2 and m + 3, of waypoint m to m + 2 (the
      // diagonal block and g of the waypoint are the top group's)
      load_step(r, q == 0, q == 0 ? nbot >= 2 : true, S, Bw, Cc, gv);
#pragma unroll
      for (int b = 0; b < NZ; ++b) S[b] = T(0);
    } else {
#pragma unroll
      for (int b = 0; b < NZ; ++b) Bw[b] = Cc[b] = T(0);
    }
    T y = T(0);
    T* rec = recs + (int64_t)r * R::SIZE;
    T* oB = on && q == 0 ? rec + R::SIZE + R::OB + a * NZ : nullptr;
    step(on, p, q == 0, q == 0 ? nbot >= 2 : true, q == 1, false, S, y, Bw, Cc, oB, nullptr);
  }
  // phase 3: the top group factors waypoints m and m + 1 with the bottom group's
  // downdates added (diagonal blocks, y, and the cross coupling H_{m+1,m})
  for (int q = 0; q < 2; ++q) {
    const bool on = mid && !half;
    const int p = m + q, r = m + q;
    T S[NZ], Bw[NZ], Cc[NZ], gv = T(0);
    if (on) {
      load_step(r, p >= 1, p >= 2, S, Bw, Cc, gv);
      damp(S);
      const int sp = (nbot + 1 - q) % 3;  // the bottom group's slot of this waypoint's downdates
#pragma unroll
      for (int b = 0; b < NZ; ++b)
        if (b <= a) S[b] += sL[sp][pg * PS + tri(a, b)];
      gv -= sY[sp][pg * RS + a];
      if (q == 1) {
        // H_{m+1,m} += (the bottom's downdate of H_{m,m+1})^T: column a of it
#pragma unroll
        for (int b = 0; b < NZ; ++b) Bw[b] += sB[pg * GS + b * RS + a];
      }
    } else {
#pragma unroll
      for (int b = 0; b < NZ; ++b) {
        S[b] = T(b == a);
        Bw[b] = Cc[b] = T(0);
      }
    }
    T y = on ? -gv : T(0);
    T* rec = recs + (int64_t)r * R::SIZE;
    T* oB = on && p >= 1 ? rec + R::OB + a * NZ : nullptr;
    step(on, p, p >= 1, p >= 2, false, true, S, y, Bw, Cc, oB, on ? rec : nullptr);
  }
  // backward: top positions k = 0 .. ntop - 1 (waypoints ntop - 1 down to 0),
  // bottom positions k - 2 (waypoints m + 2 upward); delta_t = L_tt^-T (y_t -
  // the couplings' columns times the deltas already known)
  const int K2 = Tm >= 4 ? (Tm - 1) / 2 + 2 : Tm;
  T gd = T(0);
  for (int k = 0; k < K2; ++k) {
    const int q = half ? k - 2 : k;
    const bool on = act && q >= 0 && q < (half ? nbot : ntop);
    const int t = half ? ntop + q : ntop - 1 - q;
    T* rec = recs + (int64_t)t * R::SIZE;
    const int qq = q < 0 ? 0 : q;
    const int s0 = qq % 3, s1 = (qq + 2) % 3, s2 = (qq + 1) % 3;  // slots of q, q-1, q-2
    T r = on ? rec[R::OY + a] : T(0);
    // column a of the coupling to the neighbour: top: L_{t+1,t} (record t+1, OB);
    // bottom: its own record's OB (the coupling of t - 1 to t)
    const bool h1 = half ? true : q >= 1, h2 = half ? true : q >= 2;
    if (on && h1) {
      const T* cq = (half ? rec : rec + R::SIZE) + R::OB + a;
      const T* d1 = &sY[s1][gg * RS];
#pragma unroll
      for (int b = 0; b < NZ; ++b) r -= cq[b * NZ] * d1[b];
    }
    // column a and row a of L_tt (L[c][a], c >= a; L[a][b], b <= a)
    T Lc[NZ], Lr[NZ];
    if (on) {
#pragma unroll
      for (int c = 0; c < NZ; ++c) {
        Lc[c] = c >= a ? rec[R::OL + R::lcol(a) + c - a] : T(0);
        Lr[c] = c <= a ? rec[R::OL + R::lcol(c) + a - c] : T(0);
      }
    } else {
#pragma unroll
      for (int c = 0; c < NZ; ++c) Lc[c] = Lr[c] = T(c == a);
    }
    T laa = T(1);  // this lane's pivot L[a][a], inverted once
#pragma unroll
    for (int c = 0; c < NZ; ++c)
      if (c == a) laa = Lc[c];
    const T ilaa = trcp(laa);
    // the coupling two apart, L_{t',t}^T delta_{t'} = L_tt^-1 (H_{t',t}^T delta_{t'})
    // with t' = t + 2 (top) or t - 2 (bottom): the segment blocks of record t + 2
    // (top) or t (bottom), symmetric, times delta_{t'}, then a forward substitution
    {
      T u = T(0);
      if (on && h2) {
        const T* rc = half ? rec : rec + 2 * R::SIZE;
        const T* d2 = &sY[s2][gg * RS];
        u = rc[R::OCS + sa] * d2[a & ~1] + rc[R::OCS + sa + 1] * d2[a | 1];
      }
      T acc = T(0), v = T(0);
#pragma unroll
      for (int c = 0; c < NZ; ++c) {
        if (a == c) v = (u - acc) * ilaa;
        const T vc = __shfl(v, base + c, 64);
        if (a > c) acc += Lr[c] * vc;
      }
      r -= v;
    }
    // L_tt^T delta = r
    T d = T(0);
#pragma unroll
    for (int c = NZ - 1; c >= 0; --c) {
      if (a == c) d = r * ilaa;
      const T dk = __shfl(d, base + c, 64);
      if (a < c) r -= Lc[c] * dk;
    }
    __syncthreads();
    if (inw && on) {
      sY[s0][gg * RS + a] = d;
      // the middle's deltas also seed the bottom group's backward chain, as its
      // positions -1 (waypoint m + 1) and -2 (waypoint m)
      if (!half && nbot > 0 && q < 2) sY[q == 0 ? 2 : 1][pg * RS + a] = d;
    }
    if (on) {
      rec[R::OY + a] = d;
      gd += rec[R::OG + a] * d;
    }
    __syncthreads();
  }
  // per-trajectory reductions over the 2 NZ lanes of both groups
  T gsum = T(0);
  int okall = 1;
  const int tb = j2 * 2 * NZ;
#pragma unroll
  for (int k = 0; k < 2 * NZ; ++k) {
    gsum += __shfl(gd, tb + k, 64);
    okall &= __shfl((int)ok, tb + k, 64);
  }
  if (act && half == 0 && a == 0) {
    chol_ok[traj] = okall;
    gd_out[traj] = gsum;
  }
}

// FP32 five segments: 170 VGPRs by the compiler's own choice, two waves per SIMD;
// held to three (168 VGPRs), as the register budget just allows
template <int NS, typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && NS == 5 ? 3 : 1)))
    k_traj_search(RobotT<T> rb, WeightsT<T> w, TrajArgs<T> ta, LMOpts<T> o, T* __restrict__ Z,
                  const T* __restrict__ blk, T* __restrict__ lam, const T* __restrict__ cost0,
                  const T* __restrict__ gd_in, const int32_t* __restrict__ chol_ok, int32_t* __restrict__ failed,
                  int32_t* __restrict__ trials, int list_cap) {
  constexpr int NZ = 2 * NS, NU = 3 * NS;
  using R = Rec<NS>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t traj = blockIdx.x;
  if (failed[traj]) return;
  if (!chol_ok[traj]) {
    if (threadIdx.x == 0) {
      const T l = lam[traj];
      if (!(l < o.lam_max)) failed[traj] = 2;  // z and lambda would repeat from here on
      else lam[traj] = l * T(10) < o.lam_max ? l * T(10) : o.lam_max;
    }
    return;
  }
  const TrajCtx cx = traj_ctx(ta, traj);
  const int Tn = cx.pr.Tn;
  T* s_sph = reinterpret_cast<T*>(smem_raw);
  T* s_u = s_sph + 4 * cx.pr.M;
  T* s_p = s_u + Tn * NU;
  T* s_red = s_p + Tn * 3;
  const CollList<T> cl = coll_list<NS>(s_red + 8, Tn, list_cap);
  stage_spheres(ta, cx, s_sph);
  const int t = threadIdx.x;
  const bool act = t < Tn;
  T z[NZ], dl[NZ], zt[NZ];
  if (act) {
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
      z[k] = Z[(cx.wp + t) * NZ + k];
      dl[k] = blk[(cx.wp + t) * R::SIZE + R::OY + k];
    }
  }
  __syncthreads();
  const T c0 = cost0[traj], gd = gd_in[traj];
  T alpha = T(1);
  int acc = -1, ntr = 0;
  for (int tr = 0; tr < o.ls_max; ++tr) {
#pragma unroll
    for (int k = 0; k < NZ; ++k) zt[k] = act ? z[k] + alpha * dl[k] : T(0);
    // The cost's loads of the task, the spheres and the LDS arrays go through an
    // offset that is zero but opaque to the compiler, fresh in every trial: it
    // cannot hoist them out of the trial loop and keep their values in registers
    // for all trials (that doubled this kernel's registers and halved its
    // occupancy).  An integer offset keeps every pointer's address space known.
    int z0 = 0;
    asm volatile("" : "+s"(z0));
    TrajArgs<T> tal = ta;
    tal.task += z0;
    CollList<T> cll = cl;
    cll.fr += z0;
    cll.list += z0;
    cll.cnt += z0;
    const T c = traj_cost<NS>(rb, w, tal, cx, zt, s_sph + z0, s_u + z0, s_p + z0, s_red + z0, (T*)nullptr, cll);
    ++ntr;
    if (c <= c0 + T(1e-4) * alpha * gd) {
      acc = tr;
      break;
    }
    alpha *= T(0.5);
  }
  if (acc >= 0 && act) {
#pragma unroll
    for (int k = 0; k < NZ; ++k) Z[(cx.wp + t) * NZ + k] = zt[k];
  }
  if (threadIdx.x == 0) {
    T l = lam[traj];
    if (acc == 0) l = l / T(10) > o.lam_min ? l / T(10) : o.lam_min;
    if (acc < 0) {
      if (!(l < o.lam_max)) failed[traj] = 2;  // rejected at the largest damping: a fixed point
      l = l * T(10) < o.lam_max ? l * T(10) : o.lam_max;
    }
    lam[traj] = l;
    trials[traj] += ntr;
  }
}

// The line search with its step lengths tried at once, for horizons of at most
// 64 waypoints (k_traj_search4w below: up to 128) and at most 4 trials: a workgroup of 4 TP lanes holds one
// trajectory and each slice of TP lanes (a half-wave for horizons of at most 32,
// else a wave) evaluates one trial alpha = 2^-q (q = 0 .. 3), one lane per
// waypoint; the accepted step is the first that passes in the sequential order.
// Each lane sums its own waypoint's clearance (segment-ball culls, no shared work
// list).  The sequential kernel above spends a whole wave per trial, half of it
// idle outside the clearance sums on short horizons, and about 2.7 trials per
// iteration on the trajectory workload.
template <int NS, typename T, int TP>
__global__ void __launch_bounds__(4 * TP)
    k_traj_search4(RobotT<T> rb, WeightsT<T> w, TrajArgs<T> ta, LMOpts<T> o, T* __restrict__ Z,
                   const T* __restrict__ blk, T* __restrict__ lam, const T* __restrict__ cost0,
                   const T* __restrict__ gd_in, const int32_t* __restrict__ chol_ok, int32_t* __restrict__ failed,
                   int32_t* __restrict__ trials) {
  constexpr int NZ = 2 * NS, NU = 3 * NS;
  using R = Rec<NS>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_ok[4];
  const int64_t traj = blockIdx.x;
  if (failed[traj]) return;
  if (!chol_ok[traj]) {
    if (threadIdx.x == 0) {
      const T l = lam[traj];
      if (!(l < o.lam_max)) failed[traj] = 2;  // z and lambda would repeat from here on
      else lam[traj] = l * T(10) < o.lam_max ? l * T(10) : o.lam_max;
    }
    return;
  }
  const TrajCtx cx = traj_ctx(ta, traj);
  const int Tn = cx.pr.Tn, H = Tn - 1, M = cx.pr.M;
  const int sub = (int)threadIdx.x / TP, t = (int)threadIdx.x - sub * TP;
  T* s_sph = reinterpret_cast<T*>(smem_raw);
  T* s_u = s_sph + 4 * M + sub * TP * (NU + 3);
  T* s_p = s_u + TP * NU;
  stage_spheres(ta, cx, s_sph);
  const bool act = t < Tn;
  const T alpha = T(1) / T(1 << sub);
  T zt[NZ];
  if (act) {
#pragma unroll
    for (int k = 0; k < NZ; ++k)
      zt[k] = Z[(cx.wp + t) * NZ + k] + alpha * blk[(cx.wp + t) * R::SIZE + R::OY + k];
  }
  __syncthreads();
  T cst = T(0);
  if (act) {
    T Rt[9], pt[3];
    if (M == 0) {
      fk_tip<NS>(rb, zt, Rt, pt);
      cst = bounds_cost<NS>(rb, w, zt);
    } else {
      Fwd<NS, T> f;
      WeightsT<T> wb = w;  // clearance alone here; the bounds below
      wb.sq_lim = wb.sq_curv = T(0);
      cst = config_forward<NS, T, false>(rb, wb, zt, s_sph, M, 4, 1, f) + bounds_cost<NS>(rb, w, zt);
#pragma unroll
      for (int k = 0; k < 9; ++k) Rt[k] = f.R[k];
      pt[0] = f.p[0];
      pt[1] = f.p[1];
      pt[2] = f.p[2];
    }
    if (ta.kind == CR_KIND_PATH) {
      T Tt[12], ft[3], tq[3];
      load_pose(ta, cx, t, Tt);
      cst += pose_term<T, false>(w, Rt, pt, Tt, ft, tq);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      T u[3];
      ab_to_u(zt[2 * i], zt[2 * i + 1], rb.r[i], u);
#pragma unroll
      for (int j = 0; j < 3; ++j) s_u[t * NU + 3 * i + j] = u[j];
    }
    s_p[3 * t] = pt[0];
    s_p[3 * t + 1] = pt[1];
    s_p[3 * t + 2] = pt[2];
  }
  __syncthreads();
  if (act) {
    const T idt = T(1) / w.dt, idt2 = idt * idt;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      if (t >= 1) {
        const T v = (s_u[t * NU + m] - s_u[(t - 1) * NU + m]) * idt;
        const T rr = w.sq_vel * v;
        cst += T(0.5) * rr * rr;
        if (w.has_vmax && fabs(v) > w.v_max) {
          const T hr = w.sq_lim * (fabs(v) - w.v_max);
          cst += T(0.5) * hr * hr;
        }
      }
      if (t >= 2) {
        const T a = (s_u[t * NU + m] - T(2) * s_u[(t - 1) * NU + m] + s_u[(t - 2) * NU + m]) * idt2;
        const T rr = w.sq_acc * a;
        cst += T(0.5) * rr * rr;
        if (w.has_amax && fabs(a) > w.a_max) {
          const T hr = w.sq_lim * (fabs(a) - w.a_max);
          cst += T(0.5) * hr * hr;
        }
      }
    }
    if (ta.kind == CR_KIND_TRAJ) {
      if (t >= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T rr = w.sq_len * (s_p[3 * t + c] - s_p[3 * (t - 1) + c]);
          cst += T(0.5) * rr * rr;
        }
      }
      if (t == 0 || t == H) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          T za, zb;
          load_end<NS>(ta, cx, t == 0 ? 0 : 1, i, rb.r[i], &za, &zb);
          const T ra = w.sq_eq * (zt[2 * i] - za), rb2 = w.sq_eq * (zt[2 * i + 1] - zb);
          cst += T(0.5) * (ra * ra + rb2 * rb2);
        }
      }
    }
  }
#pragma unroll
  for (int off = TP / 2; off > 0; off >>= 1) cst += __shfl_xor(cst, off, TP);
  if (t == 0) s_ok[sub] = sub < o.ls_max && cst <= cost0[traj] + T(1e-4) * alpha * gd_in[traj];
  __syncthreads();
  int acc = -1;
#pragma unroll
  for (int q = 3; q >= 0; --q)
    if (s_ok[q]) acc = q;
  if (acc == sub && act) {
#pragma unroll
    for (int k = 0; k < NZ; ++k) Z[(cx.wp + t) * NZ + k] = zt[k];
  }
  if (threadIdx.x == 0) {
    T l = lam[traj];
    if (acc == 0) l = l / T(10) > o.lam_min ? l / T(10) : o.lam_min;
    if (acc < 0) {
      if (!(l < o.lam_max)) failed[traj] = 2;  // rejected at the largest damping: a fixed point
      l = l * T(10) < o.lam_max ? l * T(10) : o.lam_max;
    }
    lam[traj] = l;
    trials[traj] += acc >= 0 ? acc + 1 : (o.ls_max < 4 ? o.ls_max : 4);
  }
}

// k_traj_search4 for horizons of 65 to 128 waypoints: each lane of a slice takes
// WPL waypoints (t, t + TP, ...).  A kernel of its own, because folding the
// waypoint loop into k_traj_search4 raised that kernel's registers from 90 to
// 161 per lane (5 waves per SIMD to 3) on the common horizons.
template <int NS, typename T, int TP, int WPL>
__global__ void __launch_bounds__(4 * TP)
    k_traj_search4w(RobotT<T> rb, WeightsT<T> w, TrajArgs<T> ta, LMOpts<T> o, T* __restrict__ Z,
                   const T* __restrict__ blk, T* __restrict__ lam, const T* __restrict__ cost0,
                   const T* __restrict__ gd_in, const int32_t* __restrict__ chol_ok, int32_t* __restrict__ failed,
                   int32_t* __restrict__ trials) {
  constexpr int NZ = 2 * NS, NU = 3 * NS;
  const int TW = ta.Tmax;  // waypoints per slice in LDS: the launch's longest horizon (<= TP * WPL)
  using R = Rec<NS>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_ok[4];
  const int64_t traj = blockIdx.x;
  if (failed[traj]) return;
  if (!chol_ok[traj]) {
    if (threadIdx.x == 0) {
      const T l = lam[traj];
      if (!(l < o.lam_max)) failed[traj] = 2;  // z and lambda would repeat from here on
      else lam[traj] = l * T(10) < o.lam_max ? l * T(10) : o.lam_max;
    }
    return;
  }
  const TrajCtx cx = traj_ctx(ta, traj);
  const int Tn = cx.pr.Tn, H = Tn - 1, M = cx.pr.M;
  const int sub = (int)threadIdx.x / TP, lane = (int)threadIdx.x - sub * TP;
  T* s_sph = reinterpret_cast<T*>(smem_raw);
  T* s_u = s_sph + 4 * M + sub * TW * (NU + 3);
  T* s_p = s_u + TW * NU;
  stage_spheres(ta, cx, s_sph);
  const T alpha = T(1) / T(1 << sub);
  // the trial point of waypoint t, formed where it is used rather than kept in
  // registers across the barriers (the same expression gives the same bits)
  auto trial = [&](int t, T* zt) {
#pragma unroll
    for (int k = 0; k < NZ; ++k) zt[k] = Z[(cx.wp + t) * NZ + k] + alpha * blk[(cx.wp + t) * R::SIZE + R::OY + k];
  };
  __syncthreads();
  T cst = T(0);
#pragma unroll
  for (int j = 0; j < WPL; ++j) {
    const int t = lane + j * TP;
    if (t >= Tn) continue;
    T zj[NZ];
    trial(t, zj);
    T Rt[9], pt[3];
    if (M == 0) {
      fk_tip<NS>(rb, zj, Rt, pt);
      cst += bounds_cost<NS>(rb, w, zj);
    } else {
      Fwd<NS, T> f;
      WeightsT<T> wb = w;  // clearance alone here; the bounds below
      wb.sq_lim = wb.sq_curv = T(0);
      cst += config_forward<NS, T, false>(rb, wb, zj, s_sph, M, 4, 1, f) + bounds_cost<NS>(rb, w, zj);
#pragma unroll
      for (int k = 0; k < 9; ++k) Rt[k] = f.R[k];
      pt[0] = f.p[0];
      pt[1] = f.p[1];
      pt[2] = f.p[2];
    }
    if (ta.kind == CR_KIND_PATH) {
      T Tt[12], ft[3], tq[3];
      load_pose(ta, cx, t, Tt);
      cst += pose_term<T, false>(w, Rt, pt, Tt, ft, tq);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      T u[3];
      ab_to_u(zj[2 * i], zj[2 * i + 1], rb.r[i], u);
#pragma unroll
      for (int c = 0; c < 3; ++c) s_u[t * NU + 3 * i + c] = u[c];
    }
    s_p[3 * t] = pt[0];
    s_p[3 * t + 1] = pt[1];
    s_p[3 * t + 2] = pt[2];
  }
  __syncthreads();
  const T idt = T(1) / w.dt, idt2 = idt * idt;
#pragma unroll
  for (int j = 0; j < WPL; ++j) {
    const int t = lane + j * TP;
    if (t >= Tn) continue;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      if (t >= 1) {
        const T v = (s_u[t * NU + m] - s_u[(t - 1) * NU + m]) * idt;
        const T rr = w.sq_vel * v;
        cst += T(0.5) * rr * rr;
        if (w.has_vmax && fabs(v) > w.v_max) {
          const T hr = w.sq_lim * (fabs(v) - w.v_max);
          cst += T(0.5) * hr * hr;
        }
      }
      if (t >= 2) {
        const T a = (s_u[t * NU + m] - T(2) * s_u[(t - 1) * NU + m] + s_u[(t - 2) * NU + m]) * idt2;
        const T rr = w.sq_acc * a;
        cst += T(0.5) * rr * rr;
        if (w.has_amax && fabs(a) > w.a_max) {
          const T hr = w.sq_lim * (fabs(a) - w.a_max);
          cst += T(0.5) * hr * hr;
        }
      }
    }
    if (ta.kind == CR_KIND_TRAJ) {
      if (t >= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T rr = w.sq_len * (s_p[3 * t + c] - s_p[3 * (t - 1) + c]);
          cst += T(0.5) * rr * rr;
        }
      }
      if (t == 0 || t == H) {
        T zj[NZ];
        trial(t, zj);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          T za, zb;
          load_end<NS>(ta, cx, t == 0 ? 0 : 1, i, rb.r[i], &za, &zb);
          const T ra = w.sq_eq * (zj[2 * i] - za), rb2 = w.sq_eq * (zj[2 * i + 1] - zb);
          cst += T(0.5) * (ra * ra + rb2 * rb2);
        }
      }
    }
  }
#pragma unroll
  for (int off = TP / 2; off > 0; off >>= 1) cst += __shfl_xor(cst, off, TP);
  if (lane == 0) s_ok[sub] = sub < o.ls_max && cst <= cost0[traj] + T(1e-4) * alpha * gd_in[traj];
  __syncthreads();
  int acc = -1;
#pragma unroll
  for (int q = 3; q >= 0; --q)
    if (s_ok[q]) acc = q;
  if (acc == sub) {
#pragma unroll
    for (int j = 0; j < WPL; ++j) {
      const int t = lane + j * TP;
      if (t < Tn) {
        T zj[NZ];
        trial(t, zj);
#pragma unroll
        for (int k = 0; k < NZ; ++k) Z[(cx.wp + t) * NZ + k] = zj[k];
      }
    }
  }
  if (threadIdx.x == 0) {
    T l = lam[traj];
    if (acc == 0) l = l / T(10) > o.lam_min ? l / T(10) : o.lam_min;
    if (acc < 0) {
      if (!(l < o.lam_max)) failed[traj] = 2;  // rejected at the largest damping: a fixed point
      l = l * T(10) < o.lam_max ? l * T(10) : o.lam_max;
    }
    lam[traj] = l;
    trials[traj] += acc >= 0 ? acc + 1 : (o.ls_max < 4 ? o.ls_max : 4);
  }
}

// Final cost and collision penalty of every trajectory (SelectTop keys, argmin).
template <int NS, typename T>
__global__ void __launch_bounds__(256)
    k_traj_eval(RobotT<T> rb, WeightsT<T> w, TrajArgs<T> ta, const T* __restrict__ Z, T* __restrict__ cost,
                T* __restrict__ pen, int32_t* __restrict__ failed, int list_cap) {
  constexpr int NZ = 2 * NS, NU = 3 * NS;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t traj = blockIdx.x;
  const TrajCtx cx = traj_ctx(ta, traj);
  const int Tn = cx.pr.Tn;
  T* s_sph = reinterpret_cast<T*>(smem_raw);
  T* s_u = s_sph + 4 * cx.pr.M;
  T* s_p = s_u + Tn * NU;
  T* s_red = s_p + Tn * 3;
  const CollList<T> cl = coll_list<NS>(s_red + 8, Tn, list_cap);
  stage_spheres(ta, cx, s_sph);
  const int t = threadIdx.x;
  T z[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) z[k] = t < Tn ? Z[(cx.wp + t) * NZ + k] : T(0);
  __syncthreads();
  T pn;
  const T c = traj_cost<NS>(rb, w, ta, cx, z, s_sph, s_u, s_p, s_red, &pn, cl);
  if (threadIdx.x == 0) {
    cost[traj] = c;
    pen[traj] = pn;
    if (!tfinite(c)) failed[traj] = 1;
  }
}

// Stage-2 candidates: copy the selected stage-1 trajectories (FP64 state); one
// workgroup per stage-2 slot (problem q, slot k).
template <int NS, typename T1>
__global__ void __launch_bounds__(64)
    k_traj_gather(TrajArgs<double> ta2, const T1* __restrict__ Z1, const int32_t* __restrict__ sel,
                  double* __restrict__ Z2, int32_t* __restrict__ failed2) {
  constexpr int NZ = 2 * NS;
  const int64_t traj2 = blockIdx.x;
  const TrajCtx cx = traj_ctx(ta2, traj2);
  const int s = sel[(int64_t)cx.s * ta2.P + cx.q];
  if (threadIdx.x == 0) failed2[traj2] = s < 0 ? 1 : 0;
  const int64_t src = cx.pr.wp0 + (int64_t)(s < 0 ? 0 : s) * cx.pr.Tn;
  for (int i = threadIdx.x; i < cx.pr.Tn * NZ; i += blockDim.x) Z2[cx.wp * NZ + i] = (double)Z1[src * NZ + i];
}

template <typename T>
__global__ void k_fill(int64_t n, T* __restrict__ x, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

template <bool MAX>
__device__ __forceinline__ double block_reduce(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(v, off, 64);
    v = MAX ? fmax(v, o) : fmin(v, o);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) s = MAX ? fmax(s, red[k]) : fmin(s, red[k]);
  return s;
}

// Argmin over candidates per problem and the FP64 assessment of the winner: one
// workgroup per problem, one lane per waypoint.
template <int NS, typename TC>
__global__ void __launch_bounds__(256)
    k_traj_finalize(RobotT<double> rb, TrajArgs<double> ta, int nf, const int32_t* __restrict__ sel,
                    const TC* __restrict__ Zc, const TC* __restrict__ costc, const int32_t* __restrict__ failedc,
                    int64_t err_ld, double* __restrict__ u_out, double* __restrict__ err_out,
                    int32_t* __restrict__ status_out) {
  constexpr int NZ = 2 * NS;
  __shared__ double red[4];
  __shared__ int s_best;
  const int64_t p = blockIdx.x;
  const int64_t P = ta.P;
  TrajCtx cx;
  cx.q = p;
  cx.pr = ta.tp[p];
  cx.s = 0;
  cx.wp = 0;
  const int Tn = cx.pr.Tn;
  const int nc = nf > 0 ? nf : cx.pr.S;
  const int64_t c0 = nf > 0 ? p * nf : cx.pr.traj0;                  // first candidate's cost index
  const int64_t w0 = nf > 0 ? nf * cx.pr.tn0 : cx.pr.wp0;            // first candidate's waypoint configuration
  const int t = threadIdx.x;
  if (t == 0) {
    int best = -1, best_seed = 0;
    double best_cost = 0.0;
    for (int k = 0; k < nc; ++k) {
      const int64_t tr = c0 + k;
      const int seed = sel ? sel[k * P + p] : k;
      const double c = (double)costc[tr];
      if (seed < 0 || failedc[tr] == 1 || !tfinite(c)) continue;
      if (best < 0 || c < best_cost || (c == best_cost && seed < best_seed)) {
        best = k;
        best_cost = c;
        best_seed = seed;
      }
    }
    s_best = best;
  }
  __syncthreads();
  const int best = s_best;
  double* const uo = u_out + cx.pr.out;
  const int64_t uld = cx.pr.out_ld, ei = cx.pr.idx;
  if (best < 0) {
    const double nan = __builtin_nan("");
    for (int m = 0; m < 3 * NS && t < Tn; ++m) uo[m * uld + t] = nan;
    if (t == 0) {
      err_out[ei] = err_out[err_ld + ei] = nan;
      status_out[ei] = CR_NONFINITE;
    }
    return;
  }
  const int64_t wb = w0 + (int64_t)best * Tn;
  double pos = 0.0, rot = 0.0, viol = 0.0, thx = 0.0, gmin = DBL_MAX;
  if (t < Tn) {
    double z[NZ];
#pragma unroll
    for (int m = 0; m < NZ; ++m) z[m] = (double)Zc[(wb + t) * NZ + m];
    const bool check = ta.kind == CR_KIND_PATH || t == 0 || t == Tn - 1;
    if (check) {
      double Rc[9], pc[3], tt[12];
      fk_tip<NS>(rb, z, Rc, pc);
      if (ta.kind == CR_KIND_PATH) {
        load_pose(ta, cx, t, tt);
      } else {
        double ze[NZ];
#pragma unroll
        for (int i = 0; i < NS; ++i) load_end<NS>(ta, cx, t == 0 ? 0 : 1, i, rb.rd[i], &ze[2 * i], &ze[2 * i + 1]);
        double Re2[9], pe2[3];
        fk_tip<NS>(rb, ze, Re2, pe2);
        for (int r = 0; r < 3; ++r) {
          for (int c = 0; c < 3; ++c) tt[4 * r + c] = Re2[3 * r + c];
          tt[4 * r + 3] = pe2[r];
        }
      }
      double dp[3] = {tt[3] - pc[0], tt[7] - pc[1], tt[11] - pc[2]};
      pos = sqrt(dot3(dp, dp));
      double Re[9], te[3];
      relative_pose(Rc, pc, tt, Re, te);
      double v[3] = {0.5 * (Re[7] - Re[5]), 0.5 * (Re[2] - Re[6]), 0.5 * (Re[3] - Re[1])};
      rot = atan2(sqrt(dot3(v, v)), 0.5 * (Re[0] + Re[4] + Re[8] - 1.0));
    }
    // bounds, zero-sum output, clearance (margin 0) of every backbone point
    double Rp[9], pp[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rp[k] = (k % 4 == 0) ? 1.0 : 0.0;
    pp[0] = pp[1] = pp[2] = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      double u[3];
      ab_to_u(z[2 * i], z[2 * i + 1], rb.rd[i], u);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        uo[(3 * i + j) * uld + t] = u[j];
        viol = fmax(viol, fabs(u[j]) - rb.umaxd[i]);
      }
      const double s = z[2 * i] * z[2 * i] + z[2 * i + 1] * z[2 * i + 1];
      thx = fmax(thx, sqrt(s) - rb.theta_maxd);
      if (cx.pr.M > 0) {
        // every point of the segment lies within L_i / 2 of its arc midpoint; only
        // the sign of the smallest clearance is reported, so spheres that cannot
        // reach the segment are skipped
        double xm[3];
        seg_point(Rp, pp, z[2 * i], z[2 * i + 1], rb.Ld[i], s, 0.5, xm);
        const double* sp = ta.sph + cx.pr.sph;
        const int64_t sld = cx.pr.sph_ld;
        for (int m = 0; m < cx.pr.M; ++m) {
          const double sx = sp[m], sy = sp[sld + m], sz = sp[2 * sld + m], rs = sp[3 * sld + m];
          const double e0 = xm[0] - sx, e1 = xm[1] - sy, e2 = xm[2] - sz;
          if (sqrt(e0 * e0 + e1 * e1 + e2 * e2) - rs - rb.rd[i] - 0.5 * rb.Ld[i] > 0.0) continue;
          for (int k = 1; k <= rb.K; ++k) {
            double x[3];
            seg_point(Rp, pp, z[2 * i], z[2 * i + 1], rb.Ld[i], s, (double)k / (double)rb.K, x);
            const double d0 = x[0] - sx, d1 = x[1] - sy, d2 = x[2] - sz;
            gmin = fmin(gmin, sqrt(d0 * d0 + d1 * d1 + d2 * d2) - rs - rb.rd[i]);
          }
        }
      }
      ArcCoef<double> c = arc_coef<double, false>(s);
      double Ri[9], di[3], q[3], Rn[9];
      seg_R_d(z[2 * i], z[2 * i + 1], rb.Ld[i], c, Ri, di);
      mv3(Rp, di, q);
      pp[0] += q[0];
      pp[1] += q[1];
      pp[2] += q[2];
      mm3(Rp, Ri, Rn);
#pragma unroll
      for (int k = 0; k < 9; ++k) Rp[k] = Rn[k];
    }
  }
  pos = block_reduce<true>(pos, red);
  rot = block_reduce<true>(rot, red);
  viol = block_reduce<true>(viol, red);
  thx = block_reduce<true>(thx, red);
  gmin = block_reduce<false>(gmin, red);
  if (t == 0) {
    int32_t st = 0;
    if (viol > 1e-6 || thx > 0.0) st |= CR_LIMIT_VIOLATION;
    if (gmin < 0.0) st |= CR_COLLISION;
    if (!(pos <= 1e-3 && rot <= 3.14159265358979323846 / 180.0)) st |= CR_NOT_CONVERGED;
    if (st == 0) st = CR_SOLVED;
    err_out[ei] = pos;
    err_out[err_ld + ei] = rot;
    status_out[ei] = st;
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct TrajWs {
  void *Z1, *blk1, *lam1, *c01, *gd1, *cost1, *pen1;
  int32_t *chol1, *fail1, *trials1, *sel;
  double *Z2, *blk2, *lam2, *c02, *gd2, *cost2, *pen2;
  int32_t *chol2, *fail2, *trials2;
  TrajProb* tp;
  SelRow* rows;
  void* cand;       // path exploration: per-waypoint IK solutions (layout of Z1)
  int32_t* okf;     // and their success flags
};

// Workspace of one path / trajectory launch (struct TrajShape): stage-1 state for
// every seed trajectory, stage-2 state for n_final trajectories per problem, the
// problem table and the SelectTop rows.
static size_t traj_ws_layout(int ns, const TrajShape& sh, int nf, int kseed, cr_dtype dt, char* base, TrajWs* w) {
  const size_t t1 = dt == CR_F64 ? 8 : 4;
  const int NZ = 2 * ns, REC = rec_size(ns);  // struct Rec
  const int64_t n1 = sh.N1, w1 = sh.W1, n2 = sh.P * (nf > 0 ? nf : 1), w2 = sh.TnSum * (nf > 0 ? nf : 1);
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t at = off;
    off += al(b);
    return base ? (void*)(base + at) : nullptr;
  };
  TrajWs x{};
  x.Z1 = take(t1 * w1 * NZ);
  x.blk1 = take(t1 * w1 * REC);
  x.lam1 = take(t1 * n1);
  x.c01 = take(t1 * n1);
  x.gd1 = take(t1 * n1);
  x.cost1 = take(t1 * n1);
  x.pen1 = take(t1 * n1);
  x.chol1 = (int32_t*)take(4 * n1);
  x.fail1 = (int32_t*)take(4 * n1);
  x.trials1 = (int32_t*)take(4 * n1);
  x.sel = (int32_t*)take(4 * n2);
  x.Z2 = (double*)take(8 * w2 * NZ);
  x.blk2 = (double*)take(8 * w2 * REC);
  x.lam2 = (double*)take(8 * n2);
  x.c02 = (double*)take(8 * n2);
  x.gd2 = (double*)take(8 * n2);
  x.cost2 = (double*)take(8 * n2);
  x.pen2 = (double*)take(8 * n2);
  x.chol2 = (int32_t*)take(4 * n2);
  x.fail2 = (int32_t*)take(4 * n2);
  x.trials2 = (int32_t*)take(4 * n2);
  x.tp = (TrajProb*)take(sizeof(TrajProb) * sh.P);
  x.rows = (SelRow*)take(sizeof(SelRow) * sh.P);
  if (kseed > 0) {
    x.cand = take(t1 * w1 * NZ);
    x.okf = (int32_t*)take(4 * w1);
  }
  if (w) *w = x;
  return off;
}

TrajShape traj_uniform_shape(int64_t P, int S, int H, int M) {
  TrajShape sh;
  sh.P = P;
  sh.N1 = P * S;
  sh.W1 = P * S * (int64_t)(H + 1);
  sh.TnSum = P * (int64_t)(H + 1);
  sh.Tmax = H + 1;
  sh.Mmax = M;
  sh.Smax = S;
  return sh;
}

size_t traj_workspace_bytes(const cr_robot& rb, const TrajShape& sh, const cr_opts& o, cr_dtype dt) {
  return traj_ws_layout(rb.n_seg, sh, o.n_final, o.k_seed, dt, nullptr, nullptr);
}

size_t traj_workspace_bytes(const cr_robot& rb, int64_t P, int S, int H, const cr_opts& o, cr_dtype dt) {
  return traj_workspace_bytes(rb, traj_uniform_shape(P, S, H, 0), o, dt);
}

// Problem table of a uniform launch (every problem: S seeds, H + 1 waypoints, the
// caller's SoA arrays of the single-problem entry points).
__global__ void k_traj_table(int kind, int64_t P, int S, int Tn, int M, int per_problem, int64_t sph_ld,
                             TrajProb* __restrict__ tp) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  TrajProb r;
  r.Tn = Tn;
  r.S = S;
  r.M = M;
  r.idx = (int32_t)q;
  r.traj0 = q * S;
  r.wp0 = q * S * (int64_t)Tn;
  r.tn0 = q * Tn;
  r.task = kind == CR_KIND_PATH ? q * Tn : q;
  r.task_ld = kind == CR_KIND_PATH ? P * Tn : P;
  r.seed = q * S * (int64_t)Tn;
  r.seed_ld = P * S * (int64_t)Tn;
  r.out = q * Tn;
  r.out_ld = P * Tn;
  r.sph = per_problem ? q * M : 0;
  r.sph_ld = sph_ld;
  tp[q] = r;
}

// SelectTop rows of a trajectory launch: candidates are whole stage-1 trajectories.
__global__ void k_traj_selrows(int64_t P, int nz, const TrajProb* __restrict__ tp, SelRow* __restrict__ rows) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  const TrajProb r = tp[q];
  SelRow s;
  s.S = r.S;
  s.nz = nz * r.Tn;
  s.kbase = r.traj0;
  s.zbase = r.wp0 * nz;
  s.zsc = (int64_t)nz * r.Tn;
  rows[q] = s;
}

template <int NS, typename T>
static size_t traj_lds(int Tn, int M, bool build) {
  const int NZ = 2 * NS;
  return sizeof(T) * (size_t)(4 * M + Tn * 3 * NS + Tn * 3 + (build ? Tn * 3 * NZ : 0) + 8);
}

static int threads_for(int Tn) { return ((Tn + 63) / 64) * 64; }

// Capacity of the clearance work list of the search / evaluation kernels (0: none)
// for a launch of nt workgroups.  The list is sized to the LDS that each workgroup
// may hold when the compute units keep the launch's workgroups resident together
// (160 KiB / workgroups per CU), but never below 13 KiB per wave (about three
// waves per SIMD, which the search kernel's registers allow anyway) nor above
// 48 KiB; at least 128 entries per wave, at most 2048.  Listed triples beyond the
// capacity are evaluated by the lane that found them.
template <int NS, typename T>
static int traj_list_cap(int Tn, int M, int64_t nt) {
  if (M <= 0) return 0;
  const size_t nwv = (size_t)threads_for(Tn) / 64;
  const size_t base = traj_lds<NS, T>(Tn, M, false) + sizeof(T) * (size_t)Tn * NS * CollList<T>::FR + 16;
  const size_t limit = 48 * 1024;
  if (base + 64 * 4 > limit) return 0;
  const size_t per_cu = nt > 256 ? (size_t)((nt + 255) / 256) : 1;
  size_t budget = 160 * 1024 / per_cu;
  if (budget < 13 * 1024 * nwv) budget = 13 * 1024 * nwv;
  if (budget > limit) budget = limit;
  size_t cap = budget > base ? (budget - base) / 4 : 0;
  if (cap < 128 * nwv) cap = 128 * nwv;
  if (cap > 2048) cap = 2048;
  const size_t pairs = (size_t)Tn * NS * M;
  if (cap > pairs) cap = pairs;
  if (cap > (limit - base) / 4) cap = (limit - base) / 4;
  return cap >= 64 ? (int)cap : 0;
}

template <int NS, typename T>
static size_t traj_lds_list(int Tn, int M, int cap) {
  size_t b = traj_lds<NS, T>(Tn, M, false);
  if (cap > 0) b += sizeof(T) * (size_t)Tn * NS * CollList<T>::FR + 16 + 4 * (size_t)cap;
  return b;
}

template <int NS>
bool traj_lds_ok(int Tmax, int Mmax) {
  return traj_lds<NS, double>(Tmax, Mmax, true) <= 64 * 1024;
}

// One LM stage (iters iterations) on the nt trajectories of ta, in type T.
template <int NS, typename T>
static cr_status traj_stage(const RobotT<T>& rb, const WeightsT<T>& w, const TrajArgs<T>& ta, int Mmax,
                            const LMOpts<T>& lo, int64_t nt, int iters, T* Z, T* blk, T* lam, T* c0, T* gd,
                            int32_t* chol, int32_t* failed, int32_t* trials, hipStream_t st) {
  const int threads = threads_for(ta.Tmax);
  const int cap = traj_list_cap<NS, T>(ta.Tmax, Mmax, nt);
  const size_t lds_b = traj_lds<NS, T>(ta.Tmax, Mmax, true), lds_s = traj_lds_list<NS, T>(ta.Tmax, Mmax, cap);
  // two trajectories per normal-equation workgroup when both fit a half-wave and
  // the launch is large enough to need several rounds of resident waves (small
  // launches, such as the FP64 refinement, keep one wave per trajectory)
  const int gb = ta.Tmax <= 32 && nt >= 4096 && 2 * lds_b <= 64 * 1024 ? 2 : 1;
  constexpr int G = 64 / (4 * NS);  // trajectories per k_traj_solve workgroup (2 NZ lanes each)
  // horizons of at most 128 waypoints and at most 4 trials: the trials at once
  // (one waypoint per lane up to 64, two beyond)
  const int tw4 = ta.Tmax <= 32 ? 32 : (ta.Tmax <= 64 ? 64 : ta.Tmax);  // k_traj_search4w: Tmax per slice
  const size_t lds_4 = sizeof(T) * (size_t)(4 * Mmax + 4 * tw4 * (3 * NS + 3));
  const bool par_search = ta.Tmax <= 128 && lo.ls_max <= 4 && lds_4 <= 64 * 1024;
  // the normal-equation kernel rewrites the same records from the same z, so the
  // autotuner may time its variants on the first iteration
  auto build = [&](int v) {
    const int occ = tune_occ(TK_TRAJ_BUILD, v);
#define CR_TB(O)                                                                                                   \
  do {                                                                                                             \
    if (gb == 2)                                                                                                   \
      hipLaunchKernelGGL((k_traj_build<NS, T, O, 2>), dim3((unsigned)((nt + 1) / 2)), dim3(64), 2 * lds_b, st, rb, w, \
                         ta, Z, blk, c0, failed, nt, (int)(lds_b / sizeof(T)));                                    \
    else                                                                                                           \
      hipLaunchKernelGGL((k_traj_build<NS, T, O, 1>), dim3((unsigned)nt), dim3(threads), lds_b, st, rb, w, ta, Z,  \
                         blk, c0, failed, nt, (int)(lds_b / sizeof(T)));                                           \
  } while (0)
    if constexpr (sizeof(T) == 4) {
      if (occ == tune_occ(TK_TRAJ_BUILD, 1)) CR_TB(tune_occ(TK_TRAJ_BUILD, 1));
      else if (occ == tune_occ(TK_TRAJ_BUILD, 2)) CR_TB(tune_occ(TK_TRAJ_BUILD, 2));
      else CR_TB(1);
    } else {
      CR_TB(1);
    }
#undef CR_TB
  };
  int vb = 0;
  for (int it = 0; it < iters; ++it) {
    bool done = false;
    if (it == 0 && sizeof(T) == 4) {
      cr_status rt = tune_choose(TK_TRAJ_BUILD, NS, CR_F32, nt * (int64_t)ta.Tmax, st, build, &vb, &done);
      if (rt != CR_OK) return rt;
    }
    if (!done) build(vb);
    hipLaunchKernelGGL((k_traj_solve<NS, T>), dim3((unsigned)((nt + G - 1) / G)), dim3(64), 0, st, ta, nt, blk, lam,
                       failed, chol, gd);
    if (par_search && ta.Tmax <= 32)
      hipLaunchKernelGGL((k_traj_search4<NS, T, 32>), dim3((unsigned)nt), dim3(128), lds_4, st, rb, w, ta, lo, Z, blk,
                         lam, c0, gd, chol, failed, trials);
    else if (par_search && ta.Tmax <= 64)
      hipLaunchKernelGGL((k_traj_search4<NS, T, 64>), dim3((unsigned)nt), dim3(256), lds_4, st, rb, w, ta, lo, Z, blk,
                         lam, c0, gd, chol, failed, trials);
    else if (par_search)
      hipLaunchKernelGGL((k_traj_search4w<NS, T, 64, 2>), dim3((unsigned)nt), dim3(256), lds_4, st, rb, w, ta, lo, Z,
                         blk, lam, c0, gd, chol, failed, trials);
    else
      hipLaunchKernelGGL((k_traj_search<NS, T>), dim3((unsigned)nt), dim3(threads), lds_s, st, rb, w, ta, lo, Z, blk,
                         lam, c0, gd, chol, failed, trials, cap);
  }
  return check_hip(hipGetLastError(), "trajectory LM stage");
}

// Two-stage solve of the problems in table tp (device), all of robot rb0 and
// kind `kind`; sh describes the launch.  Outputs go where the table says; err and
// status are indexed by the table's idx with leading dimension err_ld.
template <int NS, typename T1>
static cr_status run_traj(int kind, const cr_robot& rb0, const TrajShape& sh, const TrajProb* tp, const double* task,
                          const double* useed, const double* sph, const cr_weights& w0, const cr_opts& o,
                          double* u_out, double* err_out, int64_t err_ld, int32_t* status_out, const TrajWs& ws,
                          hipStream_t st) {
  const int64_t P = sh.P, n1 = sh.N1;
  RobotT<T1> rb1 = robot_to<T1>(rb0);
  WeightsT<T1> w1 = weights_to<T1>(w0);
  RobotT<double> rbd = robot_to<double>(rb0);
  WeightsT<double> wd = weights_to<double>(w0);
  TrajArgs<T1> ta1{kind, P, 0, sh.Tmax, tp, task, sph};
  const int threads = threads_for(sh.Tmax);
  LMOpts<T1> lo1{o.ls_max, (T1)o.lambda_min, (T1)o.lambda_max};
  if (kind == CR_KIND_PATH && o.k_seed > 0) {
    hipLaunchKernelGGL((k_path_wp_ik<NS, T1>), dim3((unsigned)n1), dim3(64), 0, st, rb1, w1, lo1, ta1, useed, o.k_seed,
                       (T1)o.lambda0, (T1*)ws.cand, ws.okf);
    hipLaunchKernelGGL((k_path_chain<NS, T1>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, ta1, n1,
                       (const T1*)ws.cand, (const int32_t*)ws.okf, (T1*)ws.Z1);
  } else {
    hipLaunchKernelGGL((k_traj_init<NS, T1>), dim3((unsigned)n1), dim3(64), 0, st, rbd, ta1, useed, (T1*)ws.Z1);
  }
  hipLaunchKernelGGL((k_fill<T1>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, n1, (T1*)ws.lam1,
                     (T1)o.lambda0);
  hipLaunchKernelGGL((k_fill<int32_t>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, n1, ws.fail1, 0);
  hipLaunchKernelGGL((k_fill<int32_t>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, n1, ws.trials1, 0);
  cr_status rc = traj_stage<NS, T1>(rb1, w1, ta1, sh.Mmax, lo1, n1, o.k_init, (T1*)ws.Z1, (T1*)ws.blk1,
                                    (T1*)ws.lam1, (T1*)ws.c01, (T1*)ws.gd1, ws.chol1, ws.fail1, ws.trials1, st);
  if (rc != CR_OK) return rc;
  const int cap1 = traj_list_cap<NS, T1>(sh.Tmax, sh.Mmax, n1);
  const size_t lds_e1 = traj_lds_list<NS, T1>(sh.Tmax, sh.Mmax, cap1);
  hipLaunchKernelGGL((k_traj_eval<NS, T1>), dim3((unsigned)n1), dim3(threads), lds_e1, st, rb1, w1, ta1,
                     (const T1*)ws.Z1, (T1*)ws.cost1, (T1*)ws.pen1, ws.fail1, cap1);
  TrajArgs<double> tad{kind, P, 0, sh.Tmax, tp, task, sph};
  if (o.n_final > 0) {
    const int nf = o.n_final;
    const int64_t n2 = P * (int64_t)nf;
    // SelectTop ranks path/trajectory candidates by their total cost
    hipLaunchKernelGGL(k_traj_selrows, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, 2 * NS, tp, ws.rows);
    rc = launch_select_strided(P, sh.Smax, 0, ws.Z1, 1, 0, ws.cost1, ws.pen1, ws.fail1, nf, o.dup_eps, ws.sel,
                               sizeof(T1) == 8 ? CR_F64 : CR_F32, st, ws.rows);
    if (rc != CR_OK) return rc;
    TrajArgs<double> ta2 = tad;
    ta2.nf = nf;
    hipLaunchKernelGGL((k_traj_gather<NS, T1>), dim3((unsigned)n2), dim3(64), 0, st, ta2, (const T1*)ws.Z1, ws.sel,
                       ws.Z2, ws.fail2);
    hipLaunchKernelGGL((k_fill<double>), dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, n2, ws.lam2, o.lambda0);
    hipLaunchKernelGGL((k_fill<int32_t>), dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, n2, ws.trials2, 0);
    LMOpts<double> lo2{o.ls_max, o.lambda_min, o.lambda_max};
    rc = traj_stage<NS, double>(rbd, wd, ta2, sh.Mmax, lo2, n2, o.k_final, ws.Z2, ws.blk2, ws.lam2, ws.c02, ws.gd2,
                                ws.chol2, ws.fail2, ws.trials2, st);
    if (rc != CR_OK) return rc;
    const int cap2 = traj_list_cap<NS, double>(sh.Tmax, sh.Mmax, n2);
    const size_t lds_e2 = traj_lds_list<NS, double>(sh.Tmax, sh.Mmax, cap2);
    hipLaunchKernelGGL((k_traj_eval<NS, double>), dim3((unsigned)n2), dim3(threads), lds_e2, st, rbd, wd, ta2,
                       (const double*)ws.Z2, ws.cost2, ws.pen2, ws.fail2, cap2);
    hipLaunchKernelGGL((k_traj_finalize<NS, double>), dim3((unsigned)P), dim3(threads), 0, st, rbd, tad, nf, ws.sel,
                       (const double*)ws.Z2, (const double*)ws.cost2, ws.fail2, err_ld, u_out, err_out, status_out);
  } else {
    hipLaunchKernelGGL((k_traj_finalize<NS, T1>), dim3((unsigned)P), dim3(threads), 0, st, rbd, tad, 0,
                       (const int32_t*)nullptr, (const T1*)ws.Z1, (const T1*)ws.cost1, ws.fail1, err_ld, u_out,
                       err_out, status_out);
  }
  return check_hip(hipGetLastError(), "trajectory solve");
}

cr_status launch_traj_assess_f32(int kind, const cr_robot& rb0, const TrajProb* row, const double* task,
                                 const double* sph, int Tn, int nf, const int32_t* sel, const float* Zc,
                                 const float* costc, const int32_t* failedc, int64_t err_ld, double* u_out,
                                 double* err_out, int32_t* status_out, hipStream_t st) {
  const RobotT<double> rbd = robot_to<double>(rb0);
  const TrajArgs<double> ta{kind, 1, 0, Tn, row, task, sph};
#define CR_ASSESS_CASE(N)                                                                                          \
  case N:                                                                                                          \
    hipLaunchKernelGGL((k_traj_finalize<N, float>), dim3(1), dim3(threads_for(Tn)), 0, st, rbd, ta, nf, sel, Zc,   \
                       costc, failedc, err_ld, u_out, err_out, status_out);                                        \
    break;
  switch (rb0.n_seg) {
    CR_ASSESS_CASE(1)
    CR_ASSESS_CASE(2)
    CR_ASSESS_CASE(3)
    CR_ASSESS_CASE(4)
    CR_ASSESS_CASE(5)
    CR_ASSESS_CASE(6)
    default:
      return fail(CR_EINVAL, "n_seg out of range");
  }
#undef CR_ASSESS_CASE
  return check_hip(hipGetLastError(), "trajectory assessment");
}

cr_status launch_traj_group(int kind, const cr_robot& rb, const TrajShape& sh, const TrajProb* tp, const double* task,
                            const double* useed, const double* sph, const cr_weights& w, const cr_opts& o,
                            double* u_out, double* err_out, int64_t err_ld, int32_t* status_out, void* wsmem,
                            cr_dtype dtype, hipStream_t st) {
  TrajWs ws;
  traj_ws_layout(rb.n_seg, sh, o.n_final, o.k_seed, dtype, (char*)wsmem, &ws);
#define CR_TRAJ_CASE(N)                                                                                              \
  case N:                                                                                                            \
    if (!traj_lds_ok<N>(sh.Tmax, sh.Mmax)) return fail(CR_EINVAL, "horizon x spheres exceed 64 KiB of LDS");         \
    return dtype == CR_F64 ? run_traj<N, double>(kind, rb, sh, tp, task, useed, sph, w, o, u_out, err_out, err_ld,   \
                                                 status_out, ws, st)                                                 \
                           : run_traj<N, float>(kind, rb, sh, tp, task, useed, sph, w, o, u_out, err_out, err_ld,    \
                                                status_out, ws, st);
  switch (rb.n_seg) {
    CR_TRAJ_CASE(1)
    CR_TRAJ_CASE(2)
    CR_TRAJ_CASE(3)
    CR_TRAJ_CASE(4)
    CR_TRAJ_CASE(5)
    CR_TRAJ_CASE(6)
    default:
      return fail(CR_EINVAL, "n_seg out of range");
  }
#undef CR_TRAJ_CASE
}

TrajProb* traj_table_slot(const cr_robot& rb, const TrajShape& sh, const cr_opts& o, cr_dtype dtype, void* wsmem) {
  TrajWs ws;
  traj_ws_layout(rb.n_seg, sh, o.n_final, o.k_seed, dtype, (char*)wsmem, &ws);
  return ws.tp;
}

cr_status launch_solve_traj(int kind, const cr_robot& rb, const cr_spheres* sp, int64_t P, int H, const double* task,
                            int S, const double* useed, const cr_weights& w, const cr_opts& o, double* u_out,
                            double* err_out, int32_t* status_out, void* wsmem, cr_dtype dtype, hipStream_t st) {
  const int M = sp ? sp->n_sph : 0;
  const TrajShape sh = traj_uniform_shape(P, S, H, M);
  TrajProb* tp = traj_table_slot(rb, sh, o, dtype, wsmem);
  hipLaunchKernelGGL(k_traj_table, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, kind, P, S, H + 1, M,
                     sp ? sp->per_problem : 0, sp ? sp->ld : (int64_t)0, tp);
  return launch_traj_group(kind, rb, sh, tp, task, useed, M > 0 ? (const double*)sp->sph : nullptr, w, o, u_out,
                           err_out, P, status_out, wsmem, dtype, st);
}

}  // namespace crk
