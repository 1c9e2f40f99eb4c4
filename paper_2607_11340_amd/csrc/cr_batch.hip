// cr_batch.hip -- uneven batches: a host scheduler over a ragged problem table.
//
// The table is split into groups of one (kind, robot); each group becomes one
// ragged launch sequence (IK: struct IkProb rows; path and trajectory: struct
// TrajProb rows) whose kernels look their problem up by seed or trajectory index.
// Within a group, problems are ordered longest-first by estimated work, so the
// first workgroups dispatched carry the longest chains (LPT list scheduling over
// the compute units).  The largest path or trajectory group goes first, then
// the IK groups (a few long launches each, whose length follows the iteration
// count rather than the work), then the small path and trajectory groups, then
// the others by estimated span (work plus an allowance for their launch chains);
// each goes to the least loaded of up to four streams forked from the caller's
// stream and joined back into it.  With
// CR_BATCH_GRAPH the whole sequence is captured once into a hipGraph and
// replayed on identical calls.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cr_internal.h"

namespace crk {
namespace {

constexpr int kStreams = 4;

struct Group {
  int kind, robot;
  std::vector<int64_t> rows;  // problem indices, longest first
  double work;
  double span;  // work plus a launch-chain allowance (stream assignment)
  int64_t P, B;               // problems; IK seeds (B) or trajectories
  TrajShape sh;
  int Smax;
  int64_t tiles;  // IK: work items of the persistent stage 1 (seed tiles)
  size_t ws_off, ws_bytes;
};

double est_work(const cr_problem& p, const cr_robot& rb, const cr_opts& o) {
  const double it = o.k_init + o.n_final * (double)o.k_final / std::max(p.S, 1);
  const double pts = p.n_sph > 0 ? 1.0 + p.n_sph * rb.pts_per_seg / 256.0 : 1.0;
  return (double)p.S * (p.H + 1) * rb.n_seg * pts * it;
}

cr_status check_table(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P,
                      const cr_opts* opts) {
  if (!robots || n_robots < 1) return fail(CR_EINVAL, "need at least one robot");
  for (int r = 0; r < n_robots; ++r) {
    cr_status rc = check_robot(&robots[r]);
    if (rc == CR_OK) rc = check_inextensible(&robots[r], "cr_solve_batch");
    if (rc != CR_OK) return rc;
  }
  if (!opts) return fail(CR_EINVAL, "opts is NULL");
  for (int k = 0; k < 3; ++k) {
    cr_status rc = check_opts(&opts[k]);
    if (rc != CR_OK) return rc;
  }
  if (P < 0 || (P > 0 && !probs)) return fail(CR_EINVAL, "bad problem table");
  for (int64_t i = 0; i < P; ++i) {
    const cr_problem& p = probs[i];
    if (p.kind < CR_KIND_IK || p.kind > CR_KIND_TRAJ) return fail(CR_EINVAL, "problem %lld: kind %d", (long long)i, p.kind);
    if (p.robot < 0 || p.robot >= n_robots) return fail(CR_EINVAL, "problem %lld: robot %d", (long long)i, p.robot);
    const int hmin = p.kind == CR_KIND_TRAJ ? 1 : 0, hmax = p.kind == CR_KIND_IK ? 0 : 255;
    if (p.H < hmin || p.H > hmax) return fail(CR_EINVAL, "problem %lld: H=%d", (long long)i, p.H);
    if (p.S < 1 || p.S > 4096) return fail(CR_EINVAL, "problem %lld: S=%d", (long long)i, p.S);
    if (p.n_sph < 0 || p.n_sph > 512) return fail(CR_EINVAL, "problem %lld: n_sph=%d", (long long)i, p.n_sph);
    if (p.task_off < 0 || p.seed_off < 0 || p.sph_off < 0 || p.out_off < 0)
      return fail(CR_EINVAL, "problem %lld: negative offset", (long long)i);
  }
  return CR_OK;
}

// Groups, their order, table rows (host) and workspace slices.
struct Plan {
  std::vector<Group> groups;
  size_t ws_bytes = 0;
  std::vector<unsigned char> tables;  // concatenated device table images
  std::vector<size_t> table_off;      // per group, into `tables`
};

cr_status make_plan(const cr_robot* robots, const cr_problem* probs, int64_t P, const cr_opts* opts, cr_dtype dtype,
                    Plan* plan) {
  std::map<std::pair<int, int>, size_t> index;
  std::vector<Group>& G = plan->groups;
  for (int64_t i = 0; i < P; ++i) {
    const auto key = std::make_pair(probs[i].kind, probs[i].robot);
    auto it = index.find(key);
    if (it == index.end()) {
      it = index.emplace(key, G.size()).first;
      Group g{};
      g.kind = probs[i].kind;
      g.robot = probs[i].robot;
      G.push_back(g);
    }
    G[it->second].rows.push_back(i);
  }
  for (Group& g : G) {
    const cr_robot& rb = robots[g.robot];
    const cr_opts& o = opts[g.kind];
    std::vector<double> wk(g.rows.size());
    g.work = 0.0;
    for (size_t k = 0; k < g.rows.size(); ++k) {
      wk[k] = est_work(probs[g.rows[k]], rb, o);
      g.work += wk[k];
    }
    std::vector<size_t> ord(g.rows.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return wk[a] > wk[b]; });
    std::vector<int64_t> rows(g.rows.size());
    for (size_t k = 0; k < ord.size(); ++k) rows[k] = g.rows[ord[k]];
    g.rows.swap(rows);
  }
  // IK groups first: each is a few long launches whose length is set by the
  // iteration count, not by its (small) work, so they start at once and overlap
  // the path and trajectory groups instead of running alone at the end
  // Path and trajectory groups: a launch chain of some hundred kernels each, so
  // even a small group lasts a while.  The largest one starts first (it would
  // otherwise end the batch alone), then the IK groups, then the groups with
  // less than half the mean work (their chains overlap the long IK launches,
  // which leave room on the chip), then the others by span: their work plus
  // half the mean group work, an allowance for the chain
  double tw = 0.0;
  int nt = 0;
  for (const Group& g : G)
    if (g.kind != CR_KIND_IK) tw += g.work, ++nt;
  for (Group& g : G) g.span = g.work + (g.kind != CR_KIND_IK && nt > 0 ? 0.5 * tw / nt : 0.0);
  const double small = nt > 0 ? 0.5 * tw / nt : 0.0;
  double wmax = 0.0;
  for (const Group& g : G)
    if (g.kind != CR_KIND_IK && g.work > wmax) wmax = g.work;
  auto rank = [&](const Group& g) {
    if (g.kind == CR_KIND_IK) return 1;
    return g.work >= wmax ? 0 : (g.work < small ? 2 : 3);
  };
  std::stable_sort(G.begin(), G.end(), [&](const Group& a, const Group& b) {
    const int ra = rank(a), rb = rank(b);
    return ra != rb ? ra < rb : a.span > b.span;
  });
  size_t off = 0;
  for (Group& g : G) {
    const cr_robot& rb = robots[g.robot];
    const cr_opts& o = opts[g.kind];
    g.P = (int64_t)g.rows.size();
    g.Smax = 1;
    const size_t toff = plan->tables.size();
    plan->table_off.push_back(toff);
    if (g.kind == CR_KIND_IK) {
      std::vector<IkProb> tab(g.P);
      int64_t seed0 = 0;
      g.tiles = 0;
      for (int64_t k = 0; k < g.P; ++k) {
        const cr_problem& p = probs[g.rows[k]];
        IkProb r{};
        r.S = p.S;
        r.M = p.n_sph;
        r.idx = (int32_t)g.rows[k];
        r.pad = (int32_t)g.tiles;  // first seed tile of the problem (persistent stage 1)
        g.tiles += (p.S + 63) / 64;
        r.seed0 = seed0;
        r.task = p.task_off;
        r.task_ld = 1;
        r.seed = p.seed_off;
        r.seed_ld = p.S;
        r.out = p.out_off;
        r.out_ld = 1;
        r.sph = p.sph_off;
        r.sph_ld = p.n_sph;
        tab[k] = r;
        seed0 += p.S;
        g.Smax = std::max(g.Smax, p.S);
      }
      g.B = seed0;
      g.ws_bytes = ik_group_workspace_bytes(rb, g.P, g.B, o, dtype);
      plan->tables.resize(toff + sizeof(IkProb) * g.P);
      std::memcpy(plan->tables.data() + toff, tab.data(), sizeof(IkProb) * g.P);
    } else {
      std::vector<TrajProb> tab(g.P);
      TrajShape sh{};
      sh.P = g.P;
      for (int64_t k = 0; k < g.P; ++k) {
        const cr_problem& p = probs[g.rows[k]];
        const int Tn = p.H + 1;
        TrajProb r{};
        r.Tn = Tn;
        r.S = p.S;
        r.M = p.n_sph;
        r.idx = (int32_t)g.rows[k];
        r.traj0 = sh.N1;
        r.wp0 = sh.W1;
        r.tn0 = sh.TnSum;
        r.task = p.task_off;
        r.task_ld = g.kind == CR_KIND_PATH ? Tn : 1;
        r.seed = p.seed_off;
        r.seed_ld = (int64_t)p.S * Tn;
        r.out = p.out_off;
        r.out_ld = Tn;
        r.sph = p.sph_off;
        r.sph_ld = p.n_sph;
        tab[k] = r;
        sh.N1 += p.S;
        sh.W1 += (int64_t)p.S * Tn;
        sh.TnSum += Tn;
        sh.Tmax = std::max(sh.Tmax, Tn);
        sh.Mmax = std::max(sh.Mmax, p.n_sph);
        sh.Smax = std::max(sh.Smax, p.S);
      }
      g.sh = sh;
      g.B = sh.N1;
      g.Smax = sh.Smax;
      g.ws_bytes = traj_workspace_bytes(rb, sh, o, dtype);
      plan->tables.resize(toff + sizeof(TrajProb) * g.P);
      std::memcpy(plan->tables.data() + toff, tab.data(), sizeof(TrajProb) * g.P);
    }
    g.ws_off = off;
    off += (g.ws_bytes + 255) & ~(size_t)255;
  }
  plan->ws_bytes = off;
  return CR_OK;
}

// Library-owned side streams (default priority), created on first use per device.
std::mutex g_mu;       // side streams
std::mutex g_call_mu;  // the pinned ring and the graph cache
std::map<int, std::vector<hipStream_t>> g_streams;

// Library-owned stream the graph sequence is captured on (captures are not
// allowed on the legacy default stream, which callers often use).
std::map<int, hipStream_t> g_capture;

cr_status capture_stream(hipStream_t* out) {
  int dev = 0;
  cr_status rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc != CR_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_capture.find(dev);
  if (it == g_capture.end()) {
    hipStream_t s;
    rc = check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    if (rc != CR_OK) return rc;
    it = g_capture.emplace(dev, s).first;
  }
  *out = it->second;
  return CR_OK;
}

cr_status side_streams(std::vector<hipStream_t>* out) {
  int dev = 0;
  cr_status rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc != CR_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  auto& v = g_streams[dev];
  while ((int)v.size() < kStreams - 1) {
    hipStream_t s;
    rc = check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    if (rc != CR_OK) return rc;
    v.push_back(s);
  }
  *out = v;
  return CR_OK;
}

// Pinned copies of the group tables.  Eager calls reuse a small ring of buffers
// guarded by events; graphs own theirs.
struct Pinned {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
Pinned g_ring[4];
int g_ring_next = 0;

cr_status pinned_copy(const Plan& plan, Pinned* pb) {
  if (pb->bytes < plan.tables.size()) {
    if (pb->ptr) {
      cr_status rc = check_hip(hipHostFree(pb->ptr), "hipHostFree");
      if (rc != CR_OK) return rc;
    }
    pb->ptr = nullptr;
    pb->bytes = 0;
    cr_status rc = check_hip(hipHostMalloc(&pb->ptr, plan.tables.size() + 64, hipHostMallocDefault), "hipHostMalloc");
    if (rc != CR_OK) return rc;
    pb->bytes = plan.tables.size() + 64;
  }
  if (!plan.tables.empty()) std::memcpy(pb->ptr, plan.tables.data(), plan.tables.size());
  return CR_OK;
}

cr_status enqueue(const cr_robot* robots, const Plan& plan, const void* pinned, const void* task, const void* u_seed,
                  const void* sph, const cr_weights* weights, const cr_opts* opts, void* u_out, void* err_out,
                  int32_t* status_out, int64_t P, char* ws, cr_dtype dtype, bool persistent, hipStream_t stream) {
  std::vector<hipStream_t> side;
  cr_status rc = side_streams(&side);
  if (rc != CR_OK) return rc;
  const int nstreams = std::min<int>(kStreams, (int)plan.groups.size());
  std::vector<hipStream_t> lanes(1, stream);
  for (int k = 1; k < nstreams; ++k) lanes.push_back(side[k - 1]);
  // fork
  hipEvent_t fork = nullptr;
  if (nstreams > 1) {
    rc = check_hip(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "hipEventCreate");
    if (rc != CR_OK) return rc;
    rc = check_hip(hipEventRecord(fork, stream), "hipEventRecord");
    for (int k = 1; k < nstreams && rc == CR_OK; ++k) rc = check_hip(hipStreamWaitEvent(lanes[k], fork, 0), "wait");
    if (rc != CR_OK) return rc;
  }
  // LPT over the streams: groups come longest first, each goes to the stream with
  // the least estimated work so far
  std::vector<double> load(nstreams, 0.0);
  for (size_t gi = 0; gi < plan.groups.size() && rc == CR_OK; ++gi) {
    const Group& g = plan.groups[gi];
    const int li = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[li] += g.span;
    hipStream_t s = lanes[li];
    char* gws = ws + g.ws_off;
    const cr_robot& rb = robots[g.robot];
    const unsigned char* src = (const unsigned char*)pinned + plan.table_off[gi];
    if (g.kind == CR_KIND_IK) {
      IkProb* tp = ik_table_slot(rb, g.P, g.B, opts[g.kind], dtype, gws);
      rc = check_hip(hipMemcpyAsync(tp, src, sizeof(IkProb) * g.P, hipMemcpyHostToDevice, s), "table upload");
      if (rc == CR_OK)
        rc = launch_ik_group(rb, g.P, g.B, g.Smax, tp, (const double*)task, (const double*)u_seed,
                             (const double*)sph, weights[g.kind], opts[g.kind], (double*)u_out, (double*)err_out, P,
                             status_out, gws, dtype, persistent, g.tiles, s);
    } else {
      TrajProb* tp = traj_table_slot(rb, g.sh, opts[g.kind], dtype, gws);
      rc = check_hip(hipMemcpyAsync(tp, src, sizeof(TrajProb) * g.P, hipMemcpyHostToDevice, s), "table upload");
      if (rc == CR_OK)
        rc = launch_traj_group(g.kind, rb, g.sh, tp, (const double*)task, (const double*)u_seed, (const double*)sph,
                               weights[g.kind], opts[g.kind], (double*)u_out, (double*)err_out, P, status_out, gws,
                               dtype, s);
    }
  }
  // join
  for (int k = 1; k < nstreams; ++k) {
    hipEvent_t j;
    cr_status r2 = check_hip(hipEventCreateWithFlags(&j, hipEventDisableTiming), "hipEventCreate");
    if (r2 == CR_OK) r2 = check_hip(hipEventRecord(j, lanes[k]), "hipEventRecord");
    if (r2 == CR_OK) r2 = check_hip(hipStreamWaitEvent(stream, j, 0), "hipStreamWaitEvent");
    if (r2 == CR_OK) r2 = check_hip(hipEventDestroy(j), "hipEventDestroy");
    if (rc == CR_OK) rc = r2;
  }
  if (fork) {
    cr_status r2 = check_hip(hipEventDestroy(fork), "hipEventDestroy");
    if (rc == CR_OK) rc = r2;
  }
  return rc;
}

// Graph cache, keyed by everything the captured sequence depends on (graphs are
// launched on the caller's stream; the capture used a library stream).
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  Pinned pinned;
};
std::map<std::string, GraphEntry> g_graphs;

std::string graph_key(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P, const void* task,
                      const void* u_seed, const void* sph, const cr_weights* weights, const cr_opts* opts,
                      const void* u_out, const void* err_out, const void* status_out, const void* ws, size_t ws_bytes,
                      cr_dtype dtype, int32_t flags, hipStream_t stream) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
  int dev = 0;
  (void)hipGetDevice(&dev);
  put(&dev, sizeof dev);
  put(&n_robots, sizeof n_robots);
  for (int r = 0; r < n_robots; ++r) put(&robots[r], sizeof(cr_robot));
  put(&P, sizeof P);
  if (P > 0) put(probs, sizeof(cr_problem) * P);
  const void* ptrs[8] = {task, u_seed, sph, u_out, err_out, status_out, ws, nullptr};
  put(ptrs, sizeof ptrs);
  put(&ws_bytes, sizeof ws_bytes);
  put(weights, sizeof(cr_weights) * 3);
  put(opts, sizeof(cr_opts) * 3);
  put(&dtype, sizeof dtype);
  put(&flags, sizeof flags);
  return k;
}

}  // namespace

size_t batch_workspace_bytes(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P,
                             const cr_opts* opts, cr_dtype dtype) {
  if (check_table(robots, n_robots, probs, P, opts) != CR_OK || check_dtype(dtype) != CR_OK) return 0;
  Plan plan;
  if (make_plan(robots, probs, P, opts, dtype, &plan) != CR_OK) return 0;
  return plan.ws_bytes > 0 ? plan.ws_bytes : 256;
}

cr_status solve_batch(const cr_robot* robots, int32_t n_robots, const cr_problem* probs, int64_t P, const void* task,
                      const void* u_seed, const void* sph, const cr_weights* weights, const cr_opts* opts,
                      void* u_out, void* err_out, int32_t* status_out, void* ws, size_t ws_bytes, cr_dtype dtype,
                      int32_t flags, hipStream_t stream) {
  cr_status rc = check_table(robots, n_robots, probs, P, opts);
  if (rc != CR_OK || (rc = check_dtype(dtype)) != CR_OK) return rc;
  if (!weights) return fail(CR_EINVAL, "weights is NULL");
  for (int k = 0; k < 3; ++k)
    if ((rc = check_weights(&weights[k])) != CR_OK) return rc;
  if (P == 0) return CR_OK;
  if (!task || !u_seed || !u_out || !err_out || !status_out) return fail(CR_EINVAL, "NULL array argument");
  for (int64_t i = 0; i < P; ++i)
    if (probs[i].n_sph > 0 && !sph) return fail(CR_EINVAL, "problem %lld has spheres but sph is NULL", (long long)i);
  const bool graph = (flags & CR_BATCH_GRAPH) != 0;
  const bool persistent = (flags & CR_BATCH_PERSISTENT) != 0;
  if (graph && !ws) return fail(CR_EINVAL, "CR_BATCH_GRAPH needs a caller workspace");
  std::lock_guard<std::mutex> lk(g_call_mu);
  if (graph) {
    const std::string key = graph_key(robots, n_robots, probs, P, task, u_seed, sph, weights, opts, u_out, err_out,
                                      status_out, ws, ws_bytes, dtype, flags, stream);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) return check_hip(hipGraphLaunch(it->second.exec, stream), "hipGraphLaunch");
  }
  Plan plan;
  if ((rc = make_plan(robots, probs, P, opts, dtype, &plan)) != CR_OK) return rc;
  const size_t need = plan.ws_bytes > 0 ? plan.ws_bytes : 256;
  void* mem = ws;
  if (ws) {
    if ((uintptr_t)ws % 256) return fail(CR_EINVAL, "workspace %p is not 256-byte aligned", ws);
    if (ws_bytes < need) return fail(CR_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  } else {
    rc = check_hip(hipMallocAsync(&mem, need, stream), "hipMallocAsync(workspace)");
    if (rc != CR_OK) return rc;
  }
  if (graph) {
    GraphEntry e;
    std::vector<hipStream_t> side;  // created before the capture starts
    if ((rc = side_streams(&side)) != CR_OK) return rc;
    hipStream_t cap;
    if ((rc = capture_stream(&cap)) != CR_OK) return rc;
    if ((rc = pinned_copy(plan, &e.pinned)) != CR_OK) return rc;
    rc = check_hip(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (rc != CR_OK) return rc;
    cr_status rc_enq = enqueue(robots, plan, e.pinned.ptr, task, u_seed, sph, weights, opts, u_out, err_out,
                               status_out, P, (char*)mem, dtype, persistent, cap);
    hipGraph_t gr = nullptr;
    rc = check_hip(hipStreamEndCapture(cap, &gr), "hipStreamEndCapture");
    if (rc_enq != CR_OK) rc = rc_enq;
    if (rc == CR_OK) rc = check_hip(hipGraphInstantiate(&e.exec, gr, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (gr) (void)hipGraphDestroy(gr);
    if (rc != CR_OK) return rc;
    const std::string key = graph_key(robots, n_robots, probs, P, task, u_seed, sph, weights, opts, u_out, err_out,
                                      status_out, ws, ws_bytes, dtype, flags, stream);
    auto ins = g_graphs.emplace(key, e).first;
    return check_hip(hipGraphLaunch(ins->second.exec, stream), "hipGraphLaunch");
  }
  Pinned& pb = g_ring[g_ring_next];
  g_ring_next = (g_ring_next + 1) % 4;
  if (pb.done) {
    rc = check_hip(hipEventSynchronize(pb.done), "hipEventSynchronize");
    if (rc != CR_OK) return rc;
  } else {
    rc = check_hip(hipEventCreateWithFlags(&pb.done, hipEventDisableTiming), "hipEventCreate");
    if (rc != CR_OK) return rc;
  }
  if ((rc = pinned_copy(plan, &pb)) != CR_OK) return rc;
  rc = enqueue(robots, plan, pb.ptr, task, u_seed, sph, weights, opts, u_out, err_out, status_out, P, (char*)mem,
               dtype, persistent, stream);
  cr_status r2 = check_hip(hipEventRecord(pb.done, stream), "hipEventRecord");
  if (rc == CR_OK) rc = r2;
  if (!ws) {
    r2 = check_hip(hipFreeAsync(mem, stream), "hipFreeAsync(workspace)");
    if (rc == CR_OK) rc = r2;
  }
  return rc;
}

}  // namespace crk
