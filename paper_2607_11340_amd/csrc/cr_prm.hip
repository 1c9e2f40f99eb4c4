// cr_prm.hip -- the exploration stage of trajectory planning (Algorithm 2): one
// probabilistic roadmap per scene, built in parallel, and batched queries that
// turn (start, goal) pairs into the initial trajectories of ParallelOptimize.
//
//   ParallelSample   SampleSeeds' draws (k_sample_seeds); a node that still
//                    collides after its attempts is discarded
//   k_prm_knn        one lane per node: the k nearest kept nodes of its problem,
//                    candidates staged through LDS 64 at a time, each lane's
//                    running list in LDS
//   k_prm_motion     one lane per (node, list slot): the straight motion to that
//                    neighbour checked at n_check interior configurations with the
//                    FP64 collision test of SampleSeeds
//   k_prm_graph      one workgroup per problem: the undirected graph in CSR form,
//                    every list sorted by node index, with the edge lengths
//   k_prm_query      one workgroup per problem: ConnectToRoadmap for both ends,
//                    Dijkstra with a workgroup-wide extract-min, ResampleLinear
//                    and the seeds
// Distances, interpolations and arc lengths use explicitly rounded FP64
// operations (never contracted into multiply-adds), so the discrete decisions
// (neighbour lists, settle order, path) follow from well-defined values.
#include <climits>

#include "cr_internal.h"

namespace crk {
namespace {

constexpr int kPrmMaxNodes = 2048;
constexpr int kPrmMaxK = 32;
constexpr int kPrmMaxCheck = 64;
constexpr int kPrmMaxP = 65535;

// squared distance of two configurations, summed in component order
template <int NC>
__device__ __forceinline__ double cfg_d2(const double* a, const double* b) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double d = __dsub_rn(a[c], b[c]);
    s = __dadd_rn(s, __dmul_rn(d, d));
  }
  return s;
}

// Does interior configuration m of the straight motion a -> b, a + t (b - a)
// with t = m / (E + 1), collide with the spheres (margin 0)?
template <int NS>
__device__ bool motion_hits(const RobotT<double>& rb, const double* a, const double* b, int m, int E,
                            const double* sph, int M, int64_t ld) {
  const double t = __ddiv_rn((double)m, (double)(E + 1));
  double z[2 * NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = __dadd_rn(a[3 * i + k], __dmul_rn(t, __dsub_rn(b[3 * i + k], a[3 * i + k])));
    u_to_ab(u[0], u[1], u[2], rb.r[i], &z[2 * i], &z[2 * i + 1]);
  }
  return penetrates<NS, double>(rb, z, sph, M, ld);
}

// (d1, i1) strictly before (d2, i2): smaller distance, then smaller index
__device__ __forceinline__ bool before(double d1, int i1, double d2, int i2) {
  return d1 < d2 || (d1 == d2 && i1 < i2);
}

// Workgroup-wide (256 lanes) minimum of (d, i) in the order above; every lane
// receives it.  rd / ri: 4 slots of LDS.
__device__ void block_argmin(double& d, int& i, double* rd, int* ri) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double d2 = __shfl_xor(d, off);
    const int i2 = __shfl_xor(i, off);
    if (before(d2, i2, d, i)) {
      d = d2;
      i = i2;
    }
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    rd[threadIdx.x >> 6] = d;
    ri[threadIdx.x >> 6] = i;
  }
  __syncthreads();
  d = rd[0];
  i = ri[0];
#pragma unroll
  for (int q = 1; q < 4; ++q)
    if (before(rd[q], ri[q], d, i)) {
      d = rd[q];
      i = ri[q];
    }
}

// k nearest kept nodes of every kept node (ParallelConnect's candidates).
// nodes [3n][B], B = P * N, column p * N + v; slot s of node v at nbr[s * B + p * N + v].
template <int NS>
__global__ void __launch_bounds__(64)
    k_prm_knn(int N, int k, int64_t B, const double* __restrict__ nodes, const int32_t* __restrict__ att,
              int32_t* __restrict__ nbr) {
  constexpr int NC = 3 * NS;
  __shared__ double tile[NC][64];
  __shared__ int tkeep[64];
  extern __shared__ double knn_lists[];  // distances [k][64], then indices [k][64]
  double* Ld = knn_lists;
  int* Li = (int*)(knn_lists + 64 * k);
  const int lane = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.y * N;
  const int i = blockIdx.x * 64 + lane;
  const bool mine = i < N && att[base + i] > 0;
  double x[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) x[c] = i < N ? nodes[c * B + base + i] : 0.0;
  for (int s = 0; s < k; ++s) {
    Ld[s * 64 + lane] = INFINITY;
    Li[s * 64 + lane] = -1;
  }
  for (int j0 = 0; j0 < N; j0 += 64) {
    __syncthreads();
    const int j = j0 + lane;
    if (j < N) {
#pragma unroll
      for (int c = 0; c < NC; ++c) tile[c][lane] = nodes[c * B + base + j];
      tkeep[lane] = att[base + j] > 0;
    } else {
      tkeep[lane] = 0;
    }
    __syncthreads();
    if (!mine) continue;
    const int cnt = min(64, N - j0);
    for (int c2 = 0; c2 < cnt; ++c2) {
      if (!tkeep[c2] || j0 + c2 == i) continue;
      double y[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) y[c] = tile[c][c2];
      const double d = cfg_d2<NC>(x, y);
      // candidates arrive in index order, so an equal distance never overtakes
      if (!(d < Ld[(k - 1) * 64 + lane])) continue;
      int pos = k - 1;
      while (pos > 0 && d < Ld[(pos - 1) * 64 + lane]) {
        Ld[pos * 64 + lane] = Ld[(pos - 1) * 64 + lane];
        Li[pos * 64 + lane] = Li[(pos - 1) * 64 + lane];
        --pos;
      }
      Ld[pos * 64 + lane] = d;
      Li[pos * 64 + lane] = j0 + c2;
    }
  }
  if (i >= N) return;
  for (int s = 0; s < k; ++s) {
    const int j = Li[s * 64 + lane];
    nbr[s * B + base + i] = mine && j >= 0 ? j : CR_PRM_NONE;
  }
}

// Collision check of every listed motion; a colliding one is re-marked -1 - j.
// The motion runs from the lower-indexed node, so both ends of an edge agree.
template <int NS>
__global__ void __launch_bounds__(256)
    k_prm_motion(RobotT<double> rb, int N, int k, int E, int64_t B, const double* __restrict__ nodes,
                 const double* __restrict__ sph, int M, int per_problem, int64_t ld, int32_t* __restrict__ nbr) {
  constexpr int NC = 3 * NS;
  const int64_t p = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= N * k) return;
  const int i = e / k, s = e - (e / k) * k;
  int32_t* slot = nbr + s * B + p * N + i;
  const int j = *slot;
  if (j < 0) return;
  const int a = min(i, j), b = max(i, j);
  double ua[NC], ub[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    ua[c] = nodes[c * B + p * N + a];
    ub[c] = nodes[c * B + p * N + b];
  }
  const double* sp = sph + (per_problem ? p * M : 0);
  for (int m = 1; m <= E; ++m)
    if (motion_hits<NS>(rb, ua, ub, m, E, sp, M, ld)) {
      *slot = -1 - j;
      return;
    }
}

// Undirected roadmap of one problem in CSR form: {v, u} is an edge when either
// lists the other with a free motion.  Problem p's lists occupy adj[p * 2kN ..],
// offsets local to that block at adj_off[p * (N + 1) + v].
template <int NS>
__global__ void __launch_bounds__(256)
    k_prm_graph(int N, int k, int64_t B, const double* __restrict__ nodes, const int32_t* __restrict__ nbr,
                int32_t* __restrict__ adj_off, int32_t* __restrict__ adj, double* __restrict__ adj_w) {
  constexpr int NC = 3 * NS;
  extern __shared__ int graph_lds[];  // deg[N], cur[N], off[N + 1], part[256]
  int* deg = graph_lds;
  int* cur = deg + N;
  int* off = cur + N;
  int* part = off + N + 1;
  const int tid = threadIdx.x;
  const int64_t p = blockIdx.x;
  const int32_t* nb = nbr + p * N;  // slot s of node v at nb[s * B + v]
  int32_t* A = adj + p * (int64_t)(2 * k) * N;
  double* W = adj_w + p * (int64_t)(2 * k) * N;
  auto lists_free = [&](int v, int u) {
    for (int s = 0; s < k; ++s)
      if (nb[s * B + v] == u) return true;
    return false;
  };
  for (int v = tid; v < N; v += 256) deg[v] = 0;
  __syncthreads();
  for (int v = tid; v < N; v += 256) {
    int nf = 0;
    for (int s = 0; s < k; ++s) {
      const int j = nb[s * B + v];
      if (j < 0) continue;
      ++nf;
      if (!lists_free(j, v)) atomicAdd(&deg[j], 1);
    }
    atomicAdd(&deg[v], nf);
  }
  __syncthreads();
  // exclusive scan of the degrees, ceil(N / 256) nodes per lane
  const int chunk = (N + 255) / 256;
  const int v0 = min(N, tid * chunk), v1 = min(N, v0 + chunk);
  int sum = 0;
  for (int v = v0; v < v1; ++v) sum += deg[v];
  part[tid] = sum;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int t = 0; t < 256; ++t) {
      const int x = part[t];
      part[t] = run;
      run += x;
    }
    off[N] = run;
  }
  __syncthreads();
  int run = part[tid];
  for (int v = v0; v < v1; ++v) {
    off[v] = run;
    run += deg[v];
  }
  __syncthreads();
  // a node's own free motions first, then those of nodes that list it
  for (int v = tid; v < N; v += 256) {
    int q = off[v];
    for (int s = 0; s < k; ++s) {
      const int j = nb[s * B + v];
      if (j >= 0) A[q++] = j;
    }
    cur[v] = q;
  }
  __syncthreads();
  for (int v = tid; v < N; v += 256)
    for (int s = 0; s < k; ++s) {
      const int j = nb[s * B + v];
      if (j >= 0 && !lists_free(j, v)) A[atomicAdd(&cur[j], 1)] = v;
    }
  __syncthreads();
  for (int v = tid; v < N; v += 256) {
    const int e0 = off[v], e1 = off[v + 1];
    for (int e = e0 + 1; e < e1; ++e) {  // insertion sort by node index
      const int x = A[e];
      int q = e;
      while (q > e0 && A[q - 1] > x) {
        A[q] = A[q - 1];
        --q;
      }
      A[q] = x;
    }
    double xv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xv[c] = nodes[c * B + p * N + v];
    for (int e = e0; e < e1; ++e) {
      double xu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) xu[c] = nodes[c * B + p * N + A[e]];
      W[e] = __dsqrt_rn(cfg_d2<NC>(xv, xu));
    }
  }
  for (int v = tid; v <= N; v += 256) adj_off[p * (N + 1) + v] = off[v];
}

// One query per problem: ConnectToRoadmap, Dijkstra, ResampleLinear, seeds.
// Nodes 0..N-1 are the roadmap, N the start and N + 1 the goal (linear: the
// roadmap is skipped and the path is the straight line).
template <int NS>
__global__ void __launch_bounds__(256)
    k_prm_query(RobotT<double> rb, int64_t P, int N, int k, int E, const double* __restrict__ nodes,
                const int32_t* __restrict__ att, const int32_t* __restrict__ adj_off, const int32_t* __restrict__ adj,
                const double* __restrict__ adj_w, const double* __restrict__ sph, int M, int per_problem, int64_t ld,
                const double* __restrict__ usg, int H, int S, const double* __restrict__ bump, int linear,
                double* __restrict__ useed, int32_t* __restrict__ npath_out, int32_t* __restrict__ path_out) {
  constexpr int NC = 3 * NS;
  const int NN = linear ? 0 : N;  // roadmap nodes taking part
  const int START = NN, GOAL = NN + 1;
  extern __shared__ double query_lds[];
  double* dist = query_lds;           // [NN + 2]
  double* gw = dist + (NN + 2);       // [NN + 2] goal distances, later the path's arc lengths
  int* pred = (int*)(gw + NN + 2);    // [NN + 2]
  int* path = pred + NN + 2;          // [NN + 2]
  unsigned char* done = (unsigned char*)(path + NN + 2);  // [NN + 2]
  __shared__ double qs[NC], qg[NC], sd2[kPrmMaxK], gd2[kPrmMaxK], rd[4];
  __shared__ int sidx[kPrmMaxK], gidx[kPrmMaxK], blk[2 * kPrmMaxK + 1], ri[4], plen_s, npath_s;
  const int tid = threadIdx.x;
  const int64_t p = blockIdx.x;
  const int64_t B = P * (int64_t)N;
  const double* sp = M > 0 ? sph + (per_problem ? p * M : 0) : nullptr;
  if (tid < NC) {
    qs[tid] = usg[tid * P + p];
    qg[tid] = usg[(NC + tid) * P + p];
  }
  __syncthreads();
  auto coords = [&](int v, double* out) {
    if (v == START) {
#pragma unroll
      for (int c = 0; c < NC; ++c) out[c] = qs[c];
    } else if (v == GOAL) {
#pragma unroll
      for (int c = 0; c < NC; ++c) out[c] = qg[c];
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) out[c] = nodes[c * B + p * N + v];
    }
  };
  const double wsg = __dsqrt_rn(cfg_d2<NC>(qs, qg));
  bool reached = false;
  if (!linear) {
    // squared distances of both ends to the kept nodes
    for (int v = tid; v < N; v += 256) {
      double y[NC];
      coords(v, y);
      const bool keep = att[p * N + v] > 0;
      dist[v] = keep ? cfg_d2<NC>(qs, y) : INFINITY;
      gw[v] = keep ? cfg_d2<NC>(qg, y) : INFINITY;
    }
    __syncthreads();
    // ConnectToRoadmap: the k nearest kept nodes of each end
    int ns = 0, ng = 0;
    for (int r = 0; r < k; ++r) {
      double bs = INFINITY, bg = INFINITY;
      int is = INT_MAX, ig = INT_MAX;
      for (int v = tid; v < N; v += 256) {
        if (before(dist[v], v, bs, is)) {
          bs = dist[v];
          is = v;
        }
        if (before(gw[v], v, bg, ig)) {
          bg = gw[v];
          ig = v;
        }
      }
      block_argmin(bs, is, rd, ri);
      block_argmin(bg, ig, rd, ri);
      if (tid == 0) {
        if (bs < INFINITY) {
          sidx[ns] = is;
          sd2[ns] = bs;
          dist[is] = INFINITY;
        }
        if (bg < INFINITY) {
          gidx[ng] = ig;
          gd2[ng] = bg;
          gw[ig] = INFINITY;
        }
      }
      ns += bs < INFINITY;
      ng += bg < INFINITY;
      __syncthreads();
    }
    // collision checks of the 2k + 1 motions: start -> node, goal -> node, start -> goal
    const int nm = ns + ng + 1;
    for (int m = tid; m < nm; m += 256) blk[m] = 0;
    __syncthreads();
    if (M > 0 && E > 0) {
      for (int item = tid; item < nm * E; item += 256) {
        const int mo = item / E, q = item - mo * E + 1;
        if (blk[mo]) continue;
        double a[NC], b[NC];
        coords(mo < ns ? START : (mo < ns + ng ? GOAL : START), a);
        coords(mo < ns ? sidx[mo] : (mo < ns + ng ? gidx[mo - ns] : GOAL), b);
        if (motion_hits<NS>(rb, a, b, q, E, sp, M, ld)) atomicOr(&blk[mo], 1);
      }
    }
    for (int v = tid; v < N + 2; v += 256) {
      dist[v] = INFINITY;
      done[v] = 0;
      pred[v] = -1;
      if (v < N) gw[v] = INFINITY;
    }
    __syncthreads();
    if (tid == 0) {
      dist[START] = 0.0;
      for (int c = 0; c < ng; ++c)
        if (!blk[ns + c]) gw[gidx[c]] = __dsqrt_rn(gd2[c]);
    }
    __syncthreads();
    const bool direct = !blk[ns + ng];
    const int32_t* ao = adj_off + p * (N + 1);
    const int32_t* A = adj + p * (int64_t)(2 * k) * N;
    const double* W = adj_w + p * (int64_t)(2 * k) * N;
    // Dijkstra: settle the unsettled node of least (distance, index)
    for (;;) {
      double bd = INFINITY;
      int bi = INT_MAX;
      for (int v = tid; v < N + 2; v += 256)
        if (!done[v] && dist[v] < INFINITY && before(dist[v], v, bd, bi)) {
          bd = dist[v];
          bi = v;
        }
      block_argmin(bd, bi, rd, ri);
      if (!(bd < INFINITY)) break;
      if (bi == GOAL) {
        reached = true;
        break;
      }
      const int u = bi;
      if (tid == 0) done[u] = 1;
      if (u == START) {
        if (tid < ns && !blk[tid]) {
          const int v = sidx[tid];
          const double cand = __dadd_rn(bd, __dsqrt_rn(sd2[tid]));
          if (cand < dist[v]) {
            dist[v] = cand;
            pred[v] = u;
          }
        }
        if (tid == ns && direct) {
          const double cand = __dadd_rn(bd, wsg);
          if (cand < dist[GOAL]) {
            dist[GOAL] = cand;
            pred[GOAL] = u;
          }
        }
      } else {
        for (int e = ao[u] + tid; e < ao[u + 1]; e += 256) {
          const int v = A[e];
          if (done[v]) continue;
          const double cand = __dadd_rn(bd, W[e]);
          if (cand < dist[v]) {
            dist[v] = cand;
            pred[v] = u;
          }
        }
        if (tid == 255 && gw[u] < INFINITY) {
          const double cand = __dadd_rn(bd, gw[u]);
          if (cand < dist[GOAL]) {
            dist[GOAL] = cand;
            pred[GOAL] = u;
          }
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid == 0) {
    int m = 0;
    if (reached) {
      for (int v = GOAL; v != START; v = pred[v]) path[m++] = v;
      path[m++] = START;
      for (int a = 0, b = m - 1; a < b; ++a, --b) {
        const int t = path[a];
        path[a] = path[b];
        path[b] = t;
      }
      for (int q = 0; q < m; ++q) gw[q] = dist[path[q]];
      npath_s = m - 2;
    } else {
      path[0] = START;
      path[1] = GOAL;
      gw[0] = 0.0;
      gw[1] = wsg;
      m = 2;
      npath_s = linear ? 0 : -1;
    }
    plen_s = m;
  }
  __syncthreads();
  const int m = plen_s - 1;
  const double sm = gw[m];
  const int Tn = H + 1;
  const int64_t BS = P * (int64_t)S * Tn;
  for (int item = tid; item < S * Tn; item += 256) {
    const int s = item / Tn, t = item - (item / Tn) * Tn;
    double q[NC];
    if (t == 0 || t == H) {
      coords(path[t == 0 ? 0 : m], q);
    } else {  // ResampleLinear: arc length s_m t / H along the path
      const double sig = __ddiv_rn(__dmul_rn(sm, (double)t), (double)H);
      int i = 1;
      while (i < m && !(sig <= gw[i])) ++i;
      const double den = __dsub_rn(gw[i], gw[i - 1]);
      const double lam = den != 0.0 ? __ddiv_rn(__dsub_rn(sig, gw[i - 1]), den) : 0.0;
      double a[NC], b[NC];
      coords(path[i - 1], a);
      coords(path[i], b);
#pragma unroll
      for (int c = 0; c < NC; ++c) q[c] = __dadd_rn(a[c], __dmul_rn(lam, __dsub_rn(b[c], a[c])));
    }
    const int64_t col = (p * S + s) * Tn + t;
    if (s > 0 && bump) {  // perturbed seed, scaled back into the tendon bounds
#pragma unroll
      for (int c = 0; c < NC; ++c) q[c] = __dadd_rn(q[c], bump[c * BS + col]);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const double peak = fmax(fabs(q[3 * i]), fmax(fabs(q[3 * i + 1]), fabs(q[3 * i + 2])));
        const double f = fmin(1.0, __ddiv_rn(rb.umax[i], fmax(peak, 1e-300)));
#pragma unroll
        for (int j = 0; j < 3; ++j) q[3 * i + j] = __dmul_rn(q[3 * i + j], f);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) useed[c * BS + col] = q[c];
  }
  if (tid == 0) npath_out[p] = npath_s;
  if (path_out)
    for (int t = tid; t < N + 2; t += 256) {
      int v = -1;
      if (t <= m) v = path[t] == START ? N : (path[t] == GOAL ? N + 1 : path[t]);
      path_out[t * P + p] = v;
    }
}

size_t query_lds_bytes(int NN) { return (size_t)(NN + 2) * (8 + 8 + 4 + 4 + 1); }

template <int NS>
cr_status run_prm_build(const cr_robot& rb0, const cr_spheres* sp, int64_t P, const cr_prm_opts& o, double* nodes,
                        int32_t* att, int32_t* nbr, int32_t* adj_off, int32_t* adj, double* adj_w, hipStream_t st) {
  const RobotT<double> rb = robot_to<double>(rb0);
  const int N = o.n_nodes, k = o.k, E = o.n_check;
  const int64_t B = P * (int64_t)N;
  cr_status rc = launch_sample_seeds(rb0, sp, P, N, o.key0, o.key1, o.max_attempts, nodes, att, st);
  if (rc != CR_OK) return rc;
  hipLaunchKernelGGL((k_prm_knn<NS>), dim3((unsigned)((N + 63) / 64), (unsigned)P), dim3(64),
                     (size_t)k * 64 * (sizeof(double) + sizeof(int)), st, N, k, B, nodes, att, nbr);
  if ((rc = check_hip(hipGetLastError(), "k_prm_knn")) != CR_OK) return rc;
  const int M = sp ? sp->n_sph : 0;
  if (M > 0 && E > 0) {
    hipLaunchKernelGGL((k_prm_motion<NS>), dim3((unsigned)((N * k + 255) / 256), (unsigned)P), dim3(256), 0, st, rb,
                       N, k, E, B, nodes, (const double*)sp->sph, M, sp->per_problem, sp->ld, nbr);
    if ((rc = check_hip(hipGetLastError(), "k_prm_motion")) != CR_OK) return rc;
  }
  hipLaunchKernelGGL((k_prm_graph<NS>), dim3((unsigned)P), dim3(256), (size_t)(3 * N + 1 + 256) * sizeof(int), st, N,
                     k, B, nodes, nbr, adj_off, adj, adj_w);
  return check_hip(hipGetLastError(), "k_prm_graph");
}

template <int NS>
cr_status run_prm_query(const cr_robot& rb0, const cr_spheres* sp, int64_t P, const cr_prm_opts& o,
                        const double* nodes, const int32_t* att, const int32_t* adj_off, const int32_t* adj,
                        const double* adj_w, const double* usg, int H, int S, const double* bump, int linear,
                        double* useed, int32_t* npath, int32_t* path, hipStream_t st) {
  const RobotT<double> rb = robot_to<double>(rb0);
  const int M = sp ? sp->n_sph : 0;
  hipLaunchKernelGGL((k_prm_query<NS>), dim3((unsigned)P), dim3(256), query_lds_bytes(linear ? 0 : o.n_nodes), st, rb,
                     P, o.n_nodes, o.k, o.n_check, nodes, att, adj_off, adj, adj_w,
                     M > 0 ? (const double*)sp->sph : nullptr, M, M > 0 ? sp->per_problem : 0, M > 0 ? sp->ld : 0,
                     usg, H, S, bump, linear, useed, npath, path);
  return check_hip(hipGetLastError(), "k_prm_query");
}

cr_status check_prm(const cr_robot* robot, const cr_spheres* spheres, int64_t P, const cr_prm_opts* o) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK || (rc = check_inextensible(robot, "PRM")) != CR_OK ||
      (rc = check_spheres(spheres, P)) != CR_OK)
    return rc;
  if (robot->self_collision) return fail(CR_EUNSUPPORTED, "PRM: self contact is not supported");
  if (spheres && spheres->n_poly) return fail(CR_EINVAL, "PRM: convex polytopes are not supported");
  if (!o) return fail(CR_EINVAL, "prm options are NULL");
  if (o->n_nodes < 1 || o->n_nodes > kPrmMaxNodes) return fail(CR_EINVAL, "n_nodes=%d not in 1..%d", o->n_nodes, kPrmMaxNodes);
  if (o->k < 1 || o->k > kPrmMaxK) return fail(CR_EINVAL, "k=%d not in 1..%d", o->k, kPrmMaxK);
  if (o->n_check < 0 || o->n_check > kPrmMaxCheck) return fail(CR_EINVAL, "n_check=%d not in 0..%d", o->n_check, kPrmMaxCheck);
  if (o->max_attempts < 1 || o->max_attempts > 64) return fail(CR_EINVAL, "max_attempts=%d not in 1..64", o->max_attempts);
  if (P < 0 || P > kPrmMaxP) return fail(CR_EINVAL, "P=%lld not in 0..%d", (long long)P, kPrmMaxP);
  return CR_OK;
}

}  // namespace
}  // namespace crk

using namespace crk;

#define CR_NS_SWITCH(ns, CALL)  \
  switch (ns) {                 \
    case 1: return CALL(1);     \
    case 2: return CALL(2);     \
    case 3: return CALL(3);     \
    case 4: return CALL(4);     \
    case 5: return CALL(5);     \
    case 6: return CALL(6);     \
  }                             \
  return fail(CR_EINVAL, "n_seg out of range")

extern "C" cr_status cr_prm_build(const cr_robot* robot, const cr_spheres* spheres, int64_t P, const cr_prm_opts* prm,
                                  double* nodes, int32_t* attempts, int32_t* nbr, int32_t* adj_off, int32_t* adj,
                                  double* adj_w, hipStream_t stream) {
  cr_status rc;
  if ((rc = check_prm(robot, spheres, P, prm)) != CR_OK) return rc;
  if (P == 0) return CR_OK;
  if (!nodes || !attempts || !nbr || !adj_off || !adj || !adj_w) return fail(CR_EINVAL, "NULL array argument");
#define CR_PRM_BUILD(NS) \
  run_prm_build<NS>(*robot, spheres, P, *prm, nodes, attempts, nbr, adj_off, adj, adj_w, stream)
  CR_NS_SWITCH(robot->n_seg, CR_PRM_BUILD);
#undef CR_PRM_BUILD
}

extern "C" cr_status cr_prm_query(const cr_robot* robot, const cr_spheres* spheres, int64_t P, const cr_prm_opts* prm,
                                  const double* nodes, const int32_t* attempts, const int32_t* adj_off,
                                  const int32_t* adj, const double* adj_w, const double* u_start_goal, int32_t H,
                                  int32_t S, const double* bump, int32_t linear, double* u_seed_out,
                                  int32_t* n_path_out, int32_t* path_out, hipStream_t stream) {
  cr_status rc;
  if ((rc = check_prm(robot, spheres, P, prm)) != CR_OK) return rc;
  if (linear != 0 && linear != 1) return fail(CR_EINVAL, "linear must be 0 or 1");
  if (H < 1 || H > 255) return fail(CR_EINVAL, "H=%d not in 1..255", H);
  if (S < 1 || S > 4096) return fail(CR_EINVAL, "S=%d not in 1..4096", S);
  if (P * (int64_t)S * (H + 1) > ((int64_t)1 << 31) - 1) return fail(CR_EINVAL, "batch too large");
  if (P == 0) return CR_OK;
  if (!u_start_goal || !u_seed_out || !n_path_out) return fail(CR_EINVAL, "NULL array argument");
  if (!linear && (!nodes || !attempts || !adj_off || !adj || !adj_w)) return fail(CR_EINVAL, "NULL roadmap array");
#define CR_PRM_QUERY(NS)                                                                                              \
  run_prm_query<NS>(*robot, spheres, P, *prm, nodes, attempts, adj_off, adj, adj_w, u_start_goal, H, S, bump, linear, \
                    u_seed_out, n_path_out, path_out, stream)
  CR_NS_SWITCH(robot->n_seg, CR_PRM_QUERY);
#undef CR_PRM_QUERY
}
