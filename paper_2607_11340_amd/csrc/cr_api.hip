// cr_api.hip -- the extern "C" boundary: argument validation, workspace
// handling and dispatch to the kernel launchers.  No exception crosses it.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <vector>

#include "cr_internal.h"

namespace crk {

static thread_local char g_err[512] = "";

cr_status fail(cr_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

cr_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return CR_OK;
  return fail(CR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename T>
RobotT<T> robot_to(const cr_robot& r) {
  RobotT<T> o{};
  o.n = r.n_seg;
  o.K = r.pts_per_seg;
  for (int i = 0; i < CR_MAX_SEG; ++i) {
    o.L[i] = (T)(i < r.n_seg ? r.L[i] : 0.0);
    o.r[i] = (T)(i < r.n_seg ? r.r[i] : 1.0);
    o.umax[i] = (T)(i < r.n_seg ? r.u_max[i] : 0.0);
  }
  o.theta_max = (T)r.theta_max;
  for (int i = 0; i < CR_MAX_SEG; ++i) {
    o.Ld[i] = i < r.n_seg ? r.L[i] : 0.0;
    o.rd[i] = i < r.n_seg ? r.r[i] : 1.0;
    o.umaxd[i] = i < r.n_seg ? r.u_max[i] : 0.0;
  }
  o.theta_maxd = r.theta_max;
  o.ext = r.extensible ? 1 : 0;
  o.self = r.self_collision ? 1 : 0;
  for (int i = 0; i < CR_MAX_SEG; ++i) {
    const bool on = r.extensible && i < r.n_seg;
    o.Lmidd[i] = on ? 0.5 * (r.L_min[i] + r.L_max[i]) : 0.0;
    o.Lhalfd[i] = on ? 0.5 * (r.L_max[i] - r.L_min[i]) : 0.0;
    o.Lmid[i] = (T)o.Lmidd[i];
    o.Lhalf[i] = (T)o.Lhalfd[i];
  }
  return o;
}
template RobotT<float> robot_to<float>(const cr_robot&);
template RobotT<double> robot_to<double>(const cr_robot&);

template <typename T>
WeightsT<T> weights_to(const cr_weights& w) {
  WeightsT<T> o{};
  o.w_pos = (T)w.w_pos;
  o.w_rot = (T)w.w_rot;
  o.sq_lim = (T)sqrt(w.rho_lim);
  o.sq_curv = (T)sqrt(w.rho_curv);
  o.sq_coll = (T)sqrt(w.rho_coll);
  o.margin = (T)w.margin;
  o.sq_eq = (T)sqrt(w.rho_eq);
  o.sq_len = (T)sqrt(w.w_len);
  o.sq_vel = (T)sqrt(w.w_vel);
  o.sq_acc = (T)sqrt(w.w_acc);
  o.has_vmax = isfinite(w.v_max) ? 1 : 0;
  o.has_amax = isfinite(w.a_max) ? 1 : 0;
  o.v_max = (T)(o.has_vmax ? w.v_max : 0.0);
  o.a_max = (T)(o.has_amax ? w.a_max : 0.0);
  o.dt = (T)w.dt;
  o.margind = w.margin;
  return o;
}
template WeightsT<float> weights_to<float>(const cr_weights&);
template WeightsT<double> weights_to<double>(const cr_weights&);

// ---------------------------------------------------------------------------
// Stage timer (instrumentation for benchmarks; process-wide, one user at a time).
// ---------------------------------------------------------------------------

struct TimerState {
  bool on = false;
  std::vector<hipEvent_t> pool;                 // idle events
  std::vector<std::vector<hipEvent_t>> calls;   // per call: start + 4 stage ends
  std::vector<hipEvent_t> cur;
  std::mutex mu;
};
static TimerState g_timer;

static hipEvent_t timer_event() {
  hipEvent_t e = nullptr;
  if (!g_timer.pool.empty()) {
    e = g_timer.pool.back();
    g_timer.pool.pop_back();
  } else {
    (void)hipEventCreate(&e);
  }
  return e;
}

bool timer_on() { return g_timer.on; }

void timer_begin_call(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  g_timer.cur.clear();
  hipEvent_t e = timer_event();
  (void)hipEventRecord(e, st);
  g_timer.cur.push_back(e);
}

void timer_mark(int stage, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  (void)stage;
  hipEvent_t e = timer_event();
  (void)hipEventRecord(e, st);
  g_timer.cur.push_back(e);
}

void timer_end_call() {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  if (g_timer.cur.size() == 5) g_timer.calls.push_back(g_timer.cur);
  else g_timer.pool.insert(g_timer.pool.end(), g_timer.cur.begin(), g_timer.cur.end());
  g_timer.cur.clear();
}

static void timer_release_all() {
  for (auto& c : g_timer.calls) g_timer.pool.insert(g_timer.pool.end(), c.begin(), c.end());
  g_timer.calls.clear();
}

cr_status check_robot(const cr_robot* rb) {
  if (!rb) return fail(CR_EINVAL, "robot is NULL");
  if (rb->n_seg < 1 || rb->n_seg > CR_MAX_SEG) return fail(CR_EINVAL, "n_seg=%d not in 1..%d", rb->n_seg, CR_MAX_SEG);
  if (rb->pts_per_seg < 1 || rb->pts_per_seg > 1024) return fail(CR_EINVAL, "pts_per_seg=%d not in 1..1024", rb->pts_per_seg);
  for (int i = 0; i < rb->n_seg; ++i) {
    if (!(rb->L[i] > 0.0) || !isfinite(rb->L[i])) return fail(CR_EINVAL, "L[%d] must be finite and > 0", i);
    if (!(rb->r[i] > 0.0) || !isfinite(rb->r[i])) return fail(CR_EINVAL, "r[%d] must be finite and > 0", i);
    if (!(rb->u_max[i] > 0.0)) return fail(CR_EINVAL, "u_max[%d] must be > 0", i);
  }
  if (!(rb->theta_max > 0.0)) return fail(CR_EINVAL, "theta_max must be > 0");
  if (rb->extensible != 0 && rb->extensible != 1) return fail(CR_EINVAL, "extensible must be 0 or 1");
  if (rb->self_collision != 0 && rb->self_collision != 1) return fail(CR_EINVAL, "self_collision must be 0 or 1");
  for (int i = 0; rb->extensible && i < rb->n_seg; ++i)
    if (!(rb->L_min[i] > 0.0) || !(rb->L_min[i] <= rb->L[i]) || !(rb->L[i] <= rb->L_max[i]) || !isfinite(rb->L_max[i]))
      return fail(CR_EINVAL, "extensible segment %d needs 0 < L_min <= L <= L_max (finite)", i);
  return CR_OK;
}

cr_status check_inextensible(const cr_robot* rb, const char* what) {
  if (rb && rb->extensible) return fail(CR_EUNSUPPORTED, "%s: extensible segments are supported by cr_fk, "
                                                          "cr_cost_grad (IK) and cr_solve_ik only", what);
  if (rb && rb->self_collision && rb->n_seg >= 3)
    return fail(CR_EUNSUPPORTED, "%s: self contact is supported by cr_cost_grad (IK) and cr_solve_ik only", what);
  return CR_OK;
}

cr_status check_dtype(cr_dtype d) {
  if (d != CR_F32 && d != CR_F64) return fail(CR_EINVAL, "dtype %d invalid", (int)d);
  return CR_OK;
}

cr_status check_opts(const cr_opts* o) {
  if (!o) return fail(CR_EINVAL, "opts is NULL");
  if (o->n_final < 0 || o->n_final > 64) return fail(CR_EINVAL, "n_final=%d not in 0..64", o->n_final);
  if (o->k_init < 0 || o->k_final < 0 || o->k_seed < 0) return fail(CR_EINVAL, "negative iteration count");
  if (o->ls_max < 1 || o->ls_max > 8) return fail(CR_EINVAL, "ls_max=%d not in 1..8", o->ls_max);
  if (!(o->lambda0 > 0.0) || !(o->lambda_min > 0.0) || !(o->lambda_max >= o->lambda_min))
    return fail(CR_EINVAL, "invalid lambda bounds");
  if (!(o->dup_eps >= 0.0)) return fail(CR_EINVAL, "dup_eps must be >= 0");
  return CR_OK;
}

cr_status check_weights(const cr_weights* w) {
  if (!w) return fail(CR_EINVAL, "weights is NULL");
  const double v[] = {w->w_pos, w->w_rot, w->rho_lim, w->rho_curv, w->rho_coll, w->rho_eq, w->w_len, w->w_vel, w->w_acc};
  for (double x : v)
    if (!(x >= 0.0) || !isfinite(x)) return fail(CR_EINVAL, "weights must be finite and >= 0");
  if (!(w->dt > 0.0)) return fail(CR_EINVAL, "dt must be > 0");
  if (!(w->margin >= 0.0)) return fail(CR_EINVAL, "margin must be >= 0");
  return CR_OK;
}

cr_status check_spheres(const cr_spheres* spheres, int64_t P) {
  if (!spheres) return CR_OK;
  if (spheres->n_poly != 0) {
    if (spheres->n_poly < 0 || spheres->n_poly > 256) return fail(CR_EINVAL, "n_poly=%d not in 0..256", spheres->n_poly);
    if (spheres->n_planes < 1 || spheres->n_planes > 32)
      return fail(CR_EINVAL, "n_planes=%d not in 1..32", spheres->n_planes);
    if (!spheres->planes) return fail(CR_EINVAL, "obstacles->planes is NULL");
    const int64_t per = (int64_t)spheres->n_poly * spheres->n_planes;
    if (spheres->plane_ld < (spheres->per_problem ? per * P : per)) return fail(CR_EINVAL, "obstacles->plane_ld too small");
  }
  if (spheres->n_sph == 0) return CR_OK;
  if (spheres->n_sph < 0) return fail(CR_EINVAL, "n_sph < 0");
  if (spheres->n_sph > 512) return fail(CR_EINVAL, "n_sph=%d exceeds 512", spheres->n_sph);
  if (!spheres->sph) return fail(CR_EINVAL, "spheres->sph is NULL");
  const int64_t need = spheres->per_problem ? (int64_t)spheres->n_sph * P : spheres->n_sph;
  if (spheres->ld < need) return fail(CR_EINVAL, "spheres->ld too small");
  return CR_OK;
}

// convex polytopes: IK only, inextensible robots without self contact
cr_status check_poly_ok(const cr_obstacles* obst, const cr_robot* rb, bool ik, const char* who) {
  if (!obst || obst->n_poly == 0) return CR_OK;
  if (!ik) return fail(CR_EINVAL, "%s: convex polytopes are supported for IK only", who);
  if (rb && (rb->extensible || rb->self_collision))
    return fail(CR_EINVAL, "%s: convex polytopes are not supported with extensible segments or self contact", who);
  return CR_OK;
}

}  // namespace crk

using namespace crk;

extern "C" {

const char* cr_status_string(cr_status s) {
  switch (s) {
    case CR_OK:
      return "CR_OK";
    case CR_EINVAL:
      return "CR_EINVAL: invalid argument";
    case CR_ENOMEM:
      return "CR_ENOMEM: workspace too small or allocation failed";
    case CR_EDEVICE:
      return "CR_EDEVICE: HIP call failed";
    case CR_EUNSUPPORTED:
      return "CR_EUNSUPPORTED: not implemented";
  }
  return "unknown cr_status";
}

const char* cr_last_error(void) { return g_err; }

cr_status cr_fk(const cr_robot* robot, int64_t B, const void* u, int64_t ld, void* arc, void* frames, void* pts,
                cr_dtype dtype, hipStream_t stream) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK || (rc = check_dtype(dtype)) != CR_OK) return rc;
  if (B < 0 || ld < B) return fail(CR_EINVAL, "need 0 <= B <= ld (B=%lld, ld=%lld)", (long long)B, (long long)ld);
  if (B > 0 && !u) return fail(CR_EINVAL, "u is NULL");
  return launch_fk(*robot, B, u, ld, arc, frames, pts, dtype, stream);
}


size_t cr_solve_ik_workspace(const cr_robot* robot, int64_t P, int32_t S, const cr_opts* opts, cr_dtype dtype) {
  if (check_robot(robot) != CR_OK || check_opts(opts) != CR_OK || check_dtype(dtype) != CR_OK || P < 0 || S < 1)
    return 0;
  return ik_workspace_layout(*robot, P, S, *opts, dtype, nullptr, nullptr);
}

cr_status cr_solve_ik(const cr_robot* robot, const cr_spheres* spheres, int64_t P, const void* T_target, int32_t S,
                      const void* u_seed, const cr_weights* weights, const cr_opts* opts, void* u_out, void* err_out,
                      int32_t* status_out, void* ws, size_t ws_bytes, cr_dtype dtype, hipStream_t stream) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK || (rc = check_dtype(dtype)) != CR_OK || (rc = check_opts(opts)) != CR_OK ||
      (rc = check_weights(weights)) != CR_OK)
    return rc;
  if (P < 0 || S < 1 || S > 4096) return fail(CR_EINVAL, "need P >= 0 and 1 <= S <= 4096");
  if (P * (int64_t)S > ((int64_t)1 << 31) - 1) return fail(CR_EINVAL, "P*S too large");
  if (P == 0) return CR_OK;
  if (!T_target || !u_seed || !u_out || !err_out || !status_out) return fail(CR_EINVAL, "NULL array argument");
  if ((rc = check_spheres(spheres, P)) != CR_OK || (rc = check_poly_ok(spheres, robot, true, "cr_solve_ik")) != CR_OK)
    return rc;
  size_t need = ik_workspace_layout(*robot, P, S, *opts, dtype, nullptr, nullptr);
  void* mem = ws;
  if (ws) {
    if ((uintptr_t)ws % 256) return fail(CR_EINVAL, "workspace %p is not 256-byte aligned", ws);
    if (ws_bytes < need) return fail(CR_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  } else {
    rc = check_hip(hipMallocAsync(&mem, need, stream), "hipMallocAsync(workspace)");
    if (rc != CR_OK) return rc;
  }
  IkWorkspace w;
  ik_workspace_layout(*robot, P, S, *opts, dtype, (char*)mem, &w);
  const cr_spheres* sp = (spheres && (spheres->n_sph > 0 || spheres->n_poly > 0)) ? spheres : nullptr;
  rc = launch_solve_ik(*robot, sp, P, (const double*)T_target, S, (const double*)u_seed, *weights, *opts,
                       (double*)u_out, (double*)err_out, status_out, w, dtype, stream);
  if (!ws) {
    cr_status rc2 = check_hip(hipFreeAsync(mem, stream), "hipFreeAsync(workspace)");
    if (rc == CR_OK) rc = rc2;
  }
  return rc;
}

cr_status cr_sample_seeds(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t S, uint64_t key0,
                          uint64_t key1, int32_t max_attempts, double* u_out, int32_t* attempts_out,
                          hipStream_t stream) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK) return rc;
  if (P < 0 || S < 1) return fail(CR_EINVAL, "need P >= 0 and S >= 1");
  if (P > ((int64_t)1 << 40) / S) return fail(CR_EINVAL, "P * S too large");
  if (max_attempts < 1 || max_attempts > 64) return fail(CR_EINVAL, "max_attempts=%d not in 1..64", max_attempts);
  if ((rc = check_spheres(spheres, P)) != CR_OK) return rc;
  if (spheres && spheres->n_poly) return fail(CR_EINVAL, "cr_sample_seeds: convex polytopes are not supported");
  if (P == 0) return CR_OK;
  if (!u_out) return fail(CR_EINVAL, "u_out is NULL");
  return launch_sample_seeds(*robot, spheres, P, S, key0, key1, max_attempts, u_out, attempts_out, stream);
}

cr_status cr_select_top(int64_t P, int32_t S, int32_t nz, const void* z, const void* e, const void* pen,
                        const int32_t* failed, int32_t n_final, double dup_eps, int32_t* idx_out, cr_dtype dtype,
                        hipStream_t stream) {
  cr_status rc;
  if ((rc = check_dtype(dtype)) != CR_OK) return rc;
  if (P < 0 || S < 1 || S > 4096) return fail(CR_EINVAL, "need P >= 0 and 1 <= S <= 4096");
  if (nz < 0 || nz > 4096) return fail(CR_EINVAL, "nz out of range");
  if (n_final < 1 || n_final > 64) return fail(CR_EINVAL, "n_final=%d not in 1..64", n_final);
  if (!(dup_eps >= 0.0)) return fail(CR_EINVAL, "dup_eps must be >= 0");
  if (P == 0) return CR_OK;
  if ((nz > 0 && !z) || !e || !pen || !idx_out) return fail(CR_EINVAL, "NULL array argument");
  return launch_select(P, S, nz, z, e, pen, failed, n_final, dup_eps, idx_out, dtype, stream);
}


static cr_status check_traj_args(const cr_robot* robot, const cr_spheres* spheres, const cr_weights* weights,
                                 const cr_opts* opts, int64_t P, int32_t H, int32_t S, int kind, cr_dtype dtype) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK || (rc = check_dtype(dtype)) != CR_OK || (rc = check_opts(opts)) != CR_OK ||
      (rc = check_weights(weights)) != CR_OK || (rc = check_inextensible(robot, "path / trajectory solve")) != CR_OK)
    return rc;
  if (P < 0 || S < 1 || S > 4096) return fail(CR_EINVAL, "need P >= 0 and 1 <= S <= 4096");
  if (H < (kind == CR_KIND_TRAJ ? 1 : 0) || H > 255) return fail(CR_EINVAL, "H=%d out of range", H);
  if (spheres && spheres->n_poly) return fail(CR_EINVAL, "paths and trajectories: convex polytopes are not supported");
  if (P * (int64_t)S * (H + 1) > ((int64_t)1 << 31) - 1) return fail(CR_EINVAL, "batch too large");
  return check_spheres(spheres, P);
}

static cr_status solve_traj_common(int kind, const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H,
                                   const void* task, int32_t S, const void* u_seed, const cr_weights* weights,
                                   const cr_opts* opts, void* u_out, void* err_out, int32_t* status_out, void* ws,
                                   size_t ws_bytes, cr_dtype dtype, hipStream_t stream) {
  cr_status rc = check_traj_args(robot, spheres, weights, opts, P, H, S, kind, dtype);
  if (rc != CR_OK) return rc;
  if (P == 0) return CR_OK;
  if (!task || !u_seed || !u_out || !err_out || !status_out) return fail(CR_EINVAL, "NULL array argument");
  const size_t need = traj_workspace_bytes(*robot, P, S, H, *opts, dtype);
  void* mem = ws;
  if (ws) {
    if ((uintptr_t)ws % 256) return fail(CR_EINVAL, "workspace %p is not 256-byte aligned", ws);
    if (ws_bytes < need) return fail(CR_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  } else {
    rc = check_hip(hipMallocAsync(&mem, need, stream), "hipMallocAsync(workspace)");
    if (rc != CR_OK) return rc;
  }
  const cr_spheres* sp = (spheres && (spheres->n_sph > 0 || spheres->n_poly > 0)) ? spheres : nullptr;
  rc = launch_solve_traj(kind, *robot, sp, P, H, (const double*)task, S, (const double*)u_seed, *weights, *opts,
                         (double*)u_out, (double*)err_out, status_out, mem, dtype, stream);
  if (!ws) {
    cr_status rc2 = check_hip(hipFreeAsync(mem, stream), "hipFreeAsync(workspace)");
    if (rc == CR_OK) rc = rc2;
  }
  return rc;
}

cr_status cr_solve_batch(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P,
                         const void* task, const void* u_seed, const void* sph, const cr_weights* weights,
                         const cr_opts* opts, void* u_out, void* err_out, int32_t* status_out, void* ws,
                         size_t ws_bytes, cr_dtype dtype, int32_t flags, hipStream_t stream) {
  return solve_batch(robots, n_robots, probs, P, task, u_seed, sph, weights, opts, u_out, err_out, status_out, ws,
                     ws_bytes, dtype, flags, stream);
}

size_t cr_solve_batch_workspace(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P,
                                const cr_opts* opts, cr_dtype dtype) {
  return batch_workspace_bytes(robots, n_robots, probs, P, opts, dtype);
}

cr_status cr_baseline_solve_ik(const cr_robot* robot, const cr_spheres* spheres, int64_t P, const void* T_target,
                               int32_t S, const void* u_seed, const cr_weights* weights, const cr_opts* opts,
                               void* u_out, void* err_out, int32_t* status_out, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK || (rc = check_opts(opts)) != CR_OK || (rc = check_weights(weights)) != CR_OK ||
      (rc = check_inextensible(robot, "cr_baseline_solve_ik")) != CR_OK)
    return rc;
  if (P < 0 || S < 1 || S > 4096) return fail(CR_EINVAL, "need P >= 0 and 1 <= S <= 4096");
  if ((rc = check_spheres(spheres, P)) != CR_OK) return rc;
  if (spheres && spheres->n_poly) return fail(CR_EINVAL, "cr_baseline_solve_ik: convex polytopes are not supported");
  if (P == 0) return CR_OK;
  if (!T_target || !u_seed || !u_out || !err_out || !status_out) return fail(CR_EINVAL, "NULL array argument");
  const size_t need = b0_workspace_bytes(*robot, S, *opts);
  void* mem = ws;
  if (ws) {
    if ((uintptr_t)ws % 256) return fail(CR_EINVAL, "workspace %p is not 256-byte aligned", ws);
    if (ws_bytes < need) return fail(CR_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  } else {
    rc = check_hip(hipMallocAsync(&mem, need, stream), "hipMallocAsync(workspace)");
    if (rc != CR_OK) return rc;
  }
  const cr_spheres* sp = (spheres && (spheres->n_sph > 0 || spheres->n_poly > 0)) ? spheres : nullptr;
  rc = launch_b0_ik(*robot, sp, P, (const double*)T_target, S, (const double*)u_seed, *weights, *opts,
                    (double*)u_out, (double*)err_out, status_out, mem, stream);
  if (!ws) {
    cr_status rc2 = check_hip(hipFreeAsync(mem, stream), "hipFreeAsync(workspace)");
    if (rc == CR_OK) rc = rc2;
  }
  return rc;
}

static cr_status baseline_traj_common(int kind, const cr_robot* robot, const cr_spheres* spheres, int64_t P,
                                      int32_t H, const void* task, int32_t S, const void* u_seed,
                                      const cr_weights* weights, const cr_opts* opts, void* u_out, void* err_out,
                                      int32_t* status_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  cr_status rc = check_traj_args(robot, spheres, weights, opts, P, H, S, kind, CR_F32);
  if (rc != CR_OK) return rc;
  if (S > 4096) return fail(CR_EINVAL, "S=%d exceeds 4096", S);
  if (P == 0) return CR_OK;
  if (!task || !u_seed || !u_out || !err_out || !status_out) return fail(CR_EINVAL, "NULL array argument");
  const size_t need = b0_traj_workspace_bytes(*robot, S, H, *opts);
  void* mem = ws;
  if (ws) {
    if ((uintptr_t)ws % 256) return fail(CR_EINVAL, "workspace %p is not 256-byte aligned", ws);
    if (ws_bytes < need) return fail(CR_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  } else {
    rc = check_hip(hipMallocAsync(&mem, need, stream), "hipMallocAsync(workspace)");
    if (rc != CR_OK) return rc;
  }
  const cr_spheres* sp = (spheres && (spheres->n_sph > 0 || spheres->n_poly > 0)) ? spheres : nullptr;
  rc = launch_b0_traj(kind, *robot, sp, P, H, (const double*)task, S, (const double*)u_seed, *weights, *opts,
                      (double*)u_out, (double*)err_out, status_out, mem, stream);
  if (!ws) {
    cr_status rc2 = check_hip(hipFreeAsync(mem, stream), "hipFreeAsync(workspace)");
    if (rc == CR_OK) rc = rc2;
  }
  return rc;
}

cr_status cr_baseline_solve_path(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H,
                                 const void* T_ref, int32_t S, const void* u_seed, const cr_weights* weights,
                                 const cr_opts* opts, void* u_out, void* err_out, int32_t* status_out, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
  return baseline_traj_common(CR_KIND_PATH, robot, spheres, P, H, T_ref, S, u_seed, weights, opts, u_out, err_out,
                              status_out, ws, ws_bytes, stream);
}

cr_status cr_baseline_solve_traj(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H,
                                 const void* u_start_goal, int32_t S, const void* u_seed, const cr_weights* weights,
                                 const cr_opts* opts, void* u_out, void* err_out, int32_t* status_out, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
  return baseline_traj_common(CR_KIND_TRAJ, robot, spheres, P, H, u_start_goal, S, u_seed, weights, opts, u_out,
                              err_out, status_out, ws, ws_bytes, stream);
}

size_t cr_baseline_traj_workspace(const cr_robot* robot, int32_t H, int32_t S, const cr_opts* opts) {
  if (check_robot(robot) != CR_OK || check_opts(opts) != CR_OK || S < 1 || S > 4096 || H < 0 || H > 255) return 0;
  return b0_traj_workspace_bytes(*robot, S, H, *opts);
}

void cr_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  timer_release_all();
  g_timer.on = on != 0;
}

cr_status cr_timing_read(double* stage_ms, int64_t* n_calls) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  if (!stage_ms || !n_calls) return fail(CR_EINVAL, "NULL output");
  for (int k = 0; k < 4; ++k) stage_ms[k] = 0.0;
  *n_calls = (int64_t)g_timer.calls.size();
  cr_status rc = CR_OK;
  for (auto& c : g_timer.calls) {
    rc = check_hip(hipEventSynchronize(c[4]), "hipEventSynchronize");
    if (rc != CR_OK) break;
    for (int k = 0; k < 4; ++k) {
      float ms = 0.0f;
      rc = check_hip(hipEventElapsedTime(&ms, c[k], c[k + 1]), "hipEventElapsedTime");
      if (rc != CR_OK) break;
      stage_ms[k] += ms;
    }
  }
  timer_release_all();
  return rc;
}

cr_status cr_ik_flop_tally(const cr_robot* robot, const cr_weights* weights, const cr_opts* opts, int64_t n,
                           const double* T_target, const double* u_seed, double* out) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK || (rc = check_opts(opts)) != CR_OK || (rc = check_weights(weights)) != CR_OK ||
      (rc = check_inextensible(robot, "cr_ik_flop_tally")) != CR_OK)
    return rc;
  if (n < 1 || !T_target || !u_seed || !out) return fail(CR_EINVAL, "need n >= 1 and non-NULL host arrays");
  return tally_ik_dispatch(*robot, *weights, *opts, n, T_target, u_seed, out);
}

cr_status cr_solve_path(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H, const void* T_ref,
                        int32_t S, const void* u_seed, const cr_weights* weights, const cr_opts* opts, void* u_out,
                        void* err_out, int32_t* status_out, void* ws, size_t ws_bytes, cr_dtype dtype,
                        hipStream_t stream) {
  return solve_traj_common(CR_KIND_PATH, robot, spheres, P, H, T_ref, S, u_seed, weights, opts, u_out, err_out,
                           status_out, ws, ws_bytes, dtype, stream);
}

cr_status cr_solve_traj(const cr_robot* robot, const cr_spheres* spheres, int64_t P, int32_t H,
                        const void* u_start_goal, int32_t S, const void* u_seed, const cr_weights* weights,
                        const cr_opts* opts, void* u_out, void* err_out, int32_t* status_out, void* ws, size_t ws_bytes,
                        cr_dtype dtype, hipStream_t stream) {
  return solve_traj_common(CR_KIND_TRAJ, robot, spheres, P, H, u_start_goal, S, u_seed, weights, opts, u_out, err_out,
                           status_out, ws, ws_bytes, dtype, stream);
}

size_t cr_solve_traj_workspace(const cr_robot* robot, int64_t P, int32_t H, int32_t S, const cr_opts* opts,
                               cr_dtype dtype) {
  if (check_robot(robot) != CR_OK || check_opts(opts) != CR_OK || check_dtype(dtype) != CR_OK || P < 0 || S < 1 ||
      H < 0 || H > 255)
    return 0;
  return traj_workspace_bytes(*robot, P, S, H, *opts, dtype);
}

cr_status cr_cost_grad(int32_t kind, const cr_robot* robot, const cr_spheres* spheres, const cr_weights* weights,
                       int64_t P, int32_t H, int32_t S, const void* task, const void* u, void* cost, void* grad,
                       const void* grad_scale, cr_dtype dtype, hipStream_t stream) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK || (rc = check_dtype(dtype)) != CR_OK || (rc = check_weights(weights)) != CR_OK)
    return rc;
  if (kind != CR_KIND_IK && kind != CR_KIND_PATH && kind != CR_KIND_TRAJ) return fail(CR_EINVAL, "kind %d invalid", kind);
  if (kind == CR_KIND_IK && H != 0) return fail(CR_EINVAL, "IK needs H = 0");
  if (kind != CR_KIND_IK && (rc = check_inextensible(robot, "cr_cost_grad for paths and trajectories")) != CR_OK)
    return rc;
  if (kind == CR_KIND_TRAJ && H < 1) return fail(CR_EINVAL, "TRAJ needs H >= 1");
  if (H < 0 || H > 255) return fail(CR_EINVAL, "H=%d not in 0..255", H);
  if (P < 0 || S < 1) return fail(CR_EINVAL, "need P >= 0 and S >= 1");
  if (P * (int64_t)S * (H + 1) > ((int64_t)1 << 31) - 1) return fail(CR_EINVAL, "batch too large");
  if (P == 0) return CR_OK;
  if (!task || !u || !cost) return fail(CR_EINVAL, "NULL array argument");
  if ((rc = check_spheres(spheres, P)) != CR_OK ||
      (rc = check_poly_ok(spheres, robot, kind == CR_KIND_IK, "cr_cost_grad")) != CR_OK)
    return rc;
  return launch_cost_grad(kind, *robot, spheres, *weights, P, H, S, task, u, cost, grad, grad_scale, dtype, stream);
}

}  // extern "C"
