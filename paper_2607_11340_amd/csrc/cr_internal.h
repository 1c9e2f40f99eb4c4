// cr_internal.h -- launchers shared between the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include "cr_device.h"
#include "cr_solver.h"

namespace crk {

// Candidates of one SelectTop problem (ragged launches): S candidates with keys
// at kbase + c, coordinate m of candidate c at z[zbase + m * zs_m + c * zsc].
struct SelRow {
  int32_t S, nz;
  int64_t kbase, zbase, zsc;
};

// One row per problem of a path / trajectory launch (device memory).  Element
// layouts: task row r, waypoint t at task + r * task_ld + t (PATH: 12 pose rows;
// TRAJ: 6n rows of start then goal actuation, t = 0); seed row r, seed s,
// waypoint t at seed + r * seed_ld + s * Tn + t; output row r, waypoint t at
// out + r * out_ld + t; sphere m, component c at sph + c * sph_ld + m.
struct TrajProb {
  int32_t Tn, S, M, idx;    // waypoints, seeds, spheres, index of err / status
  int64_t traj0, wp0, tn0;  // first stage-1 trajectory and waypoint configuration; waypoints of earlier problems
  int64_t task, task_ld, seed, seed_ld, out, out_ld, sph, sph_ld;
};


// Records a message for cr_last_error() and returns the status.
cr_status check_robot(const cr_robot* rb);
cr_status check_dtype(cr_dtype d);
cr_status check_opts(const cr_opts* o);
cr_status check_weights(const cr_weights* w);
cr_status check_spheres(const cr_spheres* spheres, int64_t P);
cr_status check_poly_ok(const cr_obstacles* obst, const cr_robot* rb, bool ik, const char* who);
cr_status check_inextensible(const cr_robot* rb, const char* what);  // CR_EUNSUPPORTED for extensible robots
cr_status fail(cr_status s, const char* fmt, ...);
cr_status check_hip(hipError_t e, const char* what);

// Launch-variant autotuning.  A tunable kernel is compiled once per occupancy
// target (minimum waves per SIMD the register allocator must allow: more waves,
// fewer registers, possibly spills).  The variants compute the same formulas; the
// compiler may fuse different products into multiply-adds under different budgets,
// so FP32 results can differ in the last bits between variants, while each variant
// is deterministic.  With tuning enabled, the first launch of a key
// (kernel, segments, dtype, launch size rounded to a power of two, device) on a
// stream that is not being captured times every variant once with HIP events and
// caches the fastest; only kernels that may run twice on the same data are tuned.
// Each variant is timed TUNE_ROUNDS times (rounds over all variants, so that clock
// and cache drift spread evenly) and its shortest time counts, which keeps the
// choice stable between runs and machines.  Tuning drains the device first (a
// device-wide synchronisation, once per key).
// The FP64 IK stage 2 is tuned over its lanes per kept candidate instead (1, 2 or
// 4; every width takes the same decisions, so its outputs do not depend on the
// variant); untuned, it takes the width that gives every SIMD one wave.
enum TuneKernel {
  TK_IK_STAGE1 = 0,
  TK_IK_STAGE1_RAG = 1,
  TK_TRAJ_BUILD = 2,
  TK_IK_STAGE2 = 3,
  TK_IK_STAGE1_Q = 4,  // the persistent stage 1 of ragged IK groups (occupancy targets as TK_IK_STAGE1_RAG)
  TK_COUNT = 5
};
constexpr int TUNE_NV = 3;      // variants per kernel
constexpr int TUNE_ROUNDS = 3;  // timings per variant
// parameter of variant v of kernel k: the occupancy target (1 = the compiler's
// own choice), or for TK_IK_STAGE2 the lanes per candidate
constexpr int tune_occ(int k, int v) {
  return k == TK_IK_STAGE2 ? 1 << v : v == 0 ? 1 : (k == TK_TRAJ_BUILD ? (v == 1 ? 2 : 3) : (v == 1 ? 3 : 4));
}
bool tune_enabled();
int tune_forced();  // -1, or the variant every tunable kernel runs
bool stream_capturing(hipStream_t st);
int tune_lookup(int kernel, int ns, int dtype, int64_t work);  // -1: not tuned yet
void tune_store(int kernel, int ns, int dtype, int64_t work, int best, const float* ms);

// The variant to launch for this key; times all variants (launch(v) enqueues
// variant v on st) when the key is new and tuning may run, leaving the outputs of
// the fastest variant (launched last, again, when it was not the last timed).
// *done: the kernel has already run.  Errors of the timed launches are returned.
template <typename F>
cr_status tune_choose(int kernel, int ns, int dtype, int64_t work, hipStream_t st, F launch, int* variant,
                      bool* done) {
  *done = false;
  *variant = 0;
  const int forced = tune_forced();
  if (forced >= 0) {
    *variant = forced;
    return CR_OK;
  }
  if (!tune_enabled()) return CR_OK;
  const int v = tune_lookup(kernel, ns, dtype, work);
  if (v >= 0) {
    *variant = v;
    return CR_OK;
  }
  if (stream_capturing(st)) return CR_OK;
  hipEvent_t ev[TUNE_NV + 1];
  int made = 0;
  cr_status rc = CR_OK;
  for (; made <= TUNE_NV && rc == CR_OK; ++made) rc = check_hip(hipEventCreate(&ev[made]), "hipEventCreate");
  float ms[TUNE_NV] = {0.0f};
  // the device is drained first, so that the variants run alone (work already
  // queued on other streams, such as other groups of a batch, would skew them)
  if (rc == CR_OK) rc = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
  if (rc == CR_OK) launch(0);  // warm-up: first-use costs of the key's buffers and code
  for (int round = 0; round < TUNE_ROUNDS && rc == CR_OK; ++round) {
    rc = check_hip(hipEventRecord(ev[0], st), "hipEventRecord");
    for (int k = 0; k < TUNE_NV && rc == CR_OK; ++k) {
      launch(k);
      rc = check_hip(hipGetLastError(), "autotune launch");
      if (rc == CR_OK) rc = check_hip(hipEventRecord(ev[k + 1], st), "hipEventRecord");
    }
    if (rc == CR_OK) rc = check_hip(hipEventSynchronize(ev[TUNE_NV]), "hipEventSynchronize");
    for (int k = 0; k < TUNE_NV && rc == CR_OK; ++k) {
      float t = 0.0f;
      rc = check_hip(hipEventElapsedTime(&t, ev[k], ev[k + 1]), "hipEventElapsedTime");
      if (rc == CR_OK && (round == 0 || t < ms[k])) ms[k] = t;
    }
  }
  for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
  if (rc != CR_OK) return rc;
  int best = 0;
  for (int k = 1; k < TUNE_NV; ++k)
    if (ms[k] < ms[best]) best = k;
  tune_store(kernel, ns, dtype, work, best, ms);
  *variant = best;
  // the outputs must be the chosen variant's, as on every later call of the key
  *done = best == TUNE_NV - 1;
  return CR_OK;
}

template <typename T>
RobotT<T> robot_to(const cr_robot& r);
template <typename T>
WeightsT<T> weights_to(const cr_weights& w);

// SampleSeeds: zero-sum triples drawn per segment before the bounds are enforced
// by scaling
constexpr int kSeedTriples = 32;
cr_status launch_sample_seeds(const cr_robot& rb, const cr_spheres* sp, int64_t P, int32_t S, uint64_t k0,
                              uint64_t k1, int32_t max_attempts, double* u_out, int32_t* attempts_out,
                              hipStream_t st);

cr_status launch_fk(const cr_robot& rb, int64_t B, const void* u, int64_t ld, void* arc, void* frames,
                    void* pts, cr_dtype dtype, hipStream_t stream);

struct IkWorkspace {
  void* z1;         // [2n][S*P] stage-1 type
  void* e1;         // [S*P]
  void* pen1;       // [S*P]
  void* cost1;      // [S*P]
  int32_t* failed1; // [S*P]
  int32_t* trials1; // [S*P]
  int32_t* sel;     // [n_final][P]
  double* z2;       // [2n][n_final*P]
  double* cost2;    // [n_final*P]
  int32_t* failed2; // [n_final*P]
};
size_t ik_workspace_layout(const cr_robot& rb, int64_t P, int32_t S, const cr_opts& o, cr_dtype dtype,
                           char* base, IkWorkspace* ws);

cr_status launch_solve_ik(const cr_robot& rb, const cr_spheres* sp, int64_t P, const double* Tt, int32_t S,
                          const double* useed, const cr_weights& w, const cr_opts& o, double* u_out, double* err_out,
                          int32_t* status_out, const IkWorkspace& ws, cr_dtype dtype, hipStream_t st);

cr_status launch_select(int64_t P, int32_t S, int32_t nz, const void* z, const void* e, const void* pen,
                        const int32_t* failed, int32_t n_final, double dup_eps, int32_t* idx_out,
                        cr_dtype dtype, hipStream_t stream);

cr_status launch_select_strided(int64_t P, int32_t S, int32_t nz, const void* z, int64_t zs_m, int64_t zs_c,
                                const void* e, const void* pen, const int32_t* failed, int32_t n_final, double dup_eps,
                                int32_t* idx_out, cr_dtype dtype, hipStream_t st, const SelRow* rows = nullptr);

// One row per problem of a ragged IK launch (device memory): pose element c
// (3x4 row-major) at task + c * task_ld; seed row r, seed s at seed + r * seed_ld
// + s; output row r at out + r * out_ld; sphere m, component c at sph + c * sph_ld
// + m.  seed0 is the problem's first seed in the launch's stage-1 arrays.
struct IkProb {
  int32_t S, M, idx, pad;
  int64_t seed0, task, task_ld, seed, seed_ld, out, out_ld, sph, sph_ld;
};
size_t ik_group_workspace_bytes(const cr_robot& rb, int64_t P, int64_t B, const cr_opts& o, cr_dtype dtype);
IkProb* ik_table_slot(const cr_robot& rb, int64_t P, int64_t B, const cr_opts& o, cr_dtype dtype, void* wsmem);
cr_status launch_ik_group(const cr_robot& rb, int64_t P, int64_t B, int Smax, const IkProb* tp, const double* task,
                          const double* useed, const double* sph, const cr_weights& w, const cr_opts& o,
                          double* u_out, double* err_out, int64_t err_ld, int32_t* status_out, void* wsmem,
                          cr_dtype dtype, bool persistent, int64_t n_tiles, hipStream_t st);

size_t batch_workspace_bytes(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P,
                             const cr_opts* opts, cr_dtype dtype);
cr_status solve_batch(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P, const void* task,
                      const void* u_seed, const void* sph, const cr_weights* weights, const cr_opts* opts,
                      void* u_out, void* err_out, int32_t* status_out, void* ws, size_t ws_bytes, cr_dtype dtype,
                      int32_t flags, hipStream_t stream);

size_t b0_workspace_bytes(const cr_robot& rb, int S, const cr_opts& o);
size_t b0_traj_workspace_bytes(const cr_robot& rb, int S, int H, const cr_opts& o);
cr_status launch_b0_traj(int kind, const cr_robot& rb, const cr_spheres* sp, int64_t P, int H, const double* task,
                         int S, const double* useed, const cr_weights& w, const cr_opts& o, double* u_out,
                         double* err_out, int32_t* status_out, void* wsmem, hipStream_t st);
// FP64 assessment and argmin of one path / trajectory problem's FP32 candidates
// (table row `row`, candidates local to it: nf kept ones with sel, or all S).
cr_status launch_traj_assess_f32(int kind, const cr_robot& rb, const TrajProb* row, const double* task,
                                 const double* sph, int Tn, int nf, const int32_t* sel, const float* Zc,
                                 const float* costc, const int32_t* failedc, int64_t err_ld, double* u_out,
                                 double* err_out, int32_t* status_out, hipStream_t st);
cr_status launch_b0_ik(const cr_robot& rb, const cr_spheres* sp, int64_t P, const double* T, int S,
                       const double* useed, const cr_weights& w, const cr_opts& o, double* u_out, double* err_out,
                       int32_t* status_out, void* wsmem, hipStream_t st);

// Totals of a path / trajectory launch: problems, stage-1 trajectories and
// waypoint configurations, waypoints summed over problems, largest horizon + 1,
// sphere count and seed count.
struct TrajShape {
  int64_t P, N1, W1, TnSum;
  int Tmax, Mmax, Smax;
};
TrajShape traj_uniform_shape(int64_t P, int S, int H, int M);
size_t traj_workspace_bytes(const cr_robot& rb, const TrajShape& sh, const cr_opts& o, cr_dtype dt);
TrajProb* traj_table_slot(const cr_robot& rb, const TrajShape& sh, const cr_opts& o, cr_dtype dtype, void* wsmem);
cr_status launch_traj_group(int kind, const cr_robot& rb, const TrajShape& sh, const TrajProb* tp, const double* task,
                            const double* useed, const double* sph, const cr_weights& w, const cr_opts& o,
                            double* u_out, double* err_out, int64_t err_ld, int32_t* status_out, void* wsmem,
                            cr_dtype dtype, hipStream_t st);
size_t traj_workspace_bytes(const cr_robot& rb, int64_t P, int S, int H, const cr_opts& o, cr_dtype dt);
cr_status launch_solve_traj(int kind, const cr_robot& rb, const cr_spheres* sp, int64_t P, int H, const double* task,
                            int S, const double* useed, const cr_weights& w, const cr_opts& o, double* u_out,
                            double* err_out, int32_t* status_out, void* wsmem, cr_dtype dtype, hipStream_t st);

cr_status launch_cost_grad(int kind, const cr_robot& rb, const cr_spheres* sp, const cr_weights& w, int64_t P, int H,
                           int S, const void* task, const void* u, void* cost, void* grad, const void* gscale,
                           cr_dtype dtype, hipStream_t st);

cr_status tally_ik_dispatch(const cr_robot& rb, const cr_weights& w, const cr_opts& o, int64_t n, const double* T,
                            const double* u, double* out);

// Stage timer: when enabled, solve calls record HIP events on their own stream
// between their stages; marks are summed by timer_read().
bool timer_on();
void timer_begin_call(hipStream_t st);   // records the call's start mark
void timer_mark(int stage, hipStream_t st);  // records the end of `stage` (0..3)
void timer_end_call();

}  // namespace crk
