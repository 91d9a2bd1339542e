// Batched stepping of several lattices (the mesh-refinement ladder of Sec. 3,
// several meshes and seeds advanced together) and the tile-height autotuner.
//
// A batch schedule is a sequence of launches; launch t advances every
// lattice g with t < steps[g] by one step, in ONE multi-lattice kernel launch
// (plus one multi-lattice wall-closure launch when walls and gravity need
// it).  The per-lattice argument blocks of every distinct launch are built on
// the host, deduplicated and copied once to the caller's device buffer.  The
// arguments alternate with the ping-pong parity, so a run of launches repeats
// a pair; each repeated pair pattern is captured once into a hipGraph (on the
// batch's own stream) and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/lbm_pp.h"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

constexpr int kMaxTables = 64;   // distinct launch argument sets per run
constexpr int kMaxGrids = 64;
constexpr int kGraphPairs = 64;  // launch pairs per captured graph

size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct LaunchRec {
  int table = -1;       // step descriptor table (update_T group 0/1 merged by signature)
  int thermal = 0;      // energy update in this launch
  int waves = 1;        // waves per strip (2: the two-wave march, energy launches only)
  int ngrid = 0;
  int nblocks = 0;
  int wall_table = -1;  // -1: no wall-closure launch
  int wall_nblocks = 0;
};

struct SimState {
  int cur, Tcur, pcur, npart;
  int64_t step;
};

}  // namespace

struct lbm_batch {
  std::vector<lbm_ctx*> g;
  hipStream_t user = nullptr, own = nullptr;
  hipEvent_t join = nullptr, t0 = nullptr, t1 = nullptr;
  char* dev = nullptr;
  size_t bytes = 0;
  int fp32 = 0, walls = 0, wall_mode = 0;
  size_t sdesc = 0, wdesc = 0;
  std::string err;
  bool timed = false;
  int64_t launches = 0, graph_launches = 0;
  // argument tables as they are in device memory (index -> bytes, starts
  // included): a run re-uploads only the tables whose content changed
  std::vector<std::string> dtab, dwtab;
  // instantiated graphs of repeated launch pairs, keyed by the pair's launch
  // shape and length; they address the tables by index, so they stay valid
  // across runs and are replayed without another capture
  std::map<std::string, hipGraphExec_t> graphs;
  // the plan of the last lbm_batch_prepare: reused by the run that follows
  // when it asks for the same schedule from the same lattice states
  std::string plan_key;
  std::vector<LaunchRec> plan_recs;
  std::vector<SimState> plan_end;

  char* step_tab(int t) const { return dev + size_t(t) * al(kMaxGrids * sdesc); }
  char* wall_tab(int t) const {
    return dev + size_t(kMaxTables) * al(kMaxGrids * sdesc) + size_t(t) * al(kMaxGrids * wdesc);
  }
  int* starts(int t) const {
    return reinterpret_cast<int*>(dev + size_t(kMaxTables) * (al(kMaxGrids * sdesc) + al(kMaxGrids * wdesc)) +
                                  size_t(t) * al((kMaxGrids + 1) * sizeof(int)));
  }
  int* wstarts(int t) const { return starts(kMaxTables + t); }
};

static size_t batch_bytes(int fp32) {
  const size_t s = step_desc_bytes(fp32), w = wall_desc_bytes(fp32);
  return size_t(kMaxTables) * (al(kMaxGrids * s) + al(kMaxGrids * w)) +
         size_t(2 * kMaxTables) * al((kMaxGrids + 1) * sizeof(int));
}

#define BTRY(b, expr)                                                     \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      (b)->err = std::string(#expr) + ": " + hipGetErrorString(e_);       \
      return LBM_E_HIP;                                                   \
    }                                                                     \
  } while (0)

extern "C" {

lbm_status lbm_batch_bytes(int32_t precision, size_t* bytes) {
  if (!bytes || (precision != LBM_FP64 && precision != LBM_FP32_SHIFTED)) return LBM_E_INVAL;
  *bytes = batch_bytes(precision == LBM_FP32_SHIFTED);
  return LBM_OK;
}

lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int32_t n, void* dev_buf, size_t bytes,
                            void* hip_stream, lbm_batch** out) {
  if (!out || !ctxs || n < 1 || n > kMaxGrids || !dev_buf) return LBM_E_INVAL;
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return LBM_E_INVAL;
  const int fp32 = ctxs[0]->p.precision == LBM_FP32_SHIFTED, walls = ctxs[0]->p.walls;
  for (int i = 0; i < n; ++i) {
    if ((ctxs[i]->p.precision == LBM_FP32_SHIFTED) != bool(fp32) || ctxs[i]->p.walls != walls)
      return fail(ctxs[i], LBM_E_INVAL, "a batch needs one precision and one wall setting");
  }
  if (bytes < batch_bytes(fp32) || reinterpret_cast<uintptr_t>(dev_buf) % 256) return LBM_E_NOMEM;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_E_NOMEM;
  b->g.assign(ctxs, ctxs + n);
  b->user = static_cast<hipStream_t>(hip_stream);
  b->dev = static_cast<char*>(dev_buf);
  b->bytes = bytes;
  b->fp32 = fp32;
  b->walls = walls;
  b->wall_mode = 0;
  if (walls) {
    b->wall_mode = 1;
    for (int i = 0; i < n; ++i)
      if (ctxs[i]->ph.wall_mod || ctxs[i]->ph.outflow_top) b->wall_mode = 2;
  }
  b->sdesc = step_desc_bytes(fp32);
  b->wdesc = wall_desc_bytes(fp32);
  // graph capture needs a stream of its own (the caller's may be the null stream)
  hipError_t e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&b->t0);
  if (e == hipSuccess) e = hipEventCreate(&b->t1);
  if (e != hipSuccess) {
    lbm_batch_destroy(b);
    return LBM_E_HIP;
  }
  *out = b;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
  if (b->own) (void)hipStreamDestroy(b->own);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->t0) (void)hipEventDestroy(b->t0);
  if (b->t1) (void)hipEventDestroy(b->t1);
  delete b;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : ""; }

static lbm_status issue(lbm_batch* b, const LaunchRec& r, hipStream_t st) {
  if (r.wall_table >= 0)
    BTRY(b, launch_wall_multi(b->fp32, b->wall_tab(r.wall_table), b->wstarts(r.wall_table), r.ngrid,
                              r.wall_nblocks, st));
  BTRY(b, launch_step_multi(b->fp32, b->wall_mode, r.thermal, r.waves, b->step_tab(r.table),
                            b->starts(r.table), r.ngrid, r.nblocks, st));
  return LBM_OK;
}

// number of lattices of a table signature: ngrid descriptors of `desc`
// bytes followed by ngrid + 1 workgroup starts
static size_t recs_ngrid_of(const std::string& sig, size_t desc) {
  return (sig.size() - sizeof(int)) / (desc + sizeof(int));
}

// Simulate the host state machine of every lattice over the schedule, build
// the launch records and bring the argument tables in device memory up to
// date (only changed tables are copied).  end[] receives each lattice's state
// after the schedule.
static lbm_status plan_run(lbm_batch* b, const int64_t* steps, std::vector<LaunchRec>& recs,
                           std::vector<SimState>& st) {
  const int n = int(b->g.size());
  int64_t T = 0;
  for (int i = 0; i < n; ++i) {
    if (steps[i] < 0) return LBM_E_INVAL;
    if (!b->g[i]->initialized) return fail(b->g[i], LBM_E_STATE, "batch member not initialised");
    T = std::max(T, steps[i]);
  }
  st.resize(n);
  for (int i = 0; i < n; ++i) st[i] = {b->g[i]->cur, b->g[i]->Tcur, b->g[i]->pcur, b->g[i]->npart, b->g[i]->step};
  std::map<std::string, int> seen, wseen;
  std::vector<std::string> tabs, wtabs;
  recs.clear();
  recs.reserve(size_t(T) * 2);
  std::vector<char> buf(b->sdesc), wbuf(b->wdesc);
  std::vector<int> ut_t(n);
  for (int64_t t = 0; t < T; ++t) {
    // lattices active in this launch (-1: done), and whether T is updated
    for (int i = 0; i < n; ++i)
      ut_t[i] = t >= steps[i] ? -1 : int(b->g[i]->p.thermal && st[i].step >= b->g[i]->p.n_iso);
    // one record per group of equal energy-update flag and waves per strip
    // (no update; update with one wave; update with two waves)
    for (int grp = 0; grp < 3; ++grp) {
      const int thermal = grp > 0, waves = grp == 2 ? 2 : 1;
      std::string sig, wsig;
      std::vector<int> starts(1, 0), wstarts(1, 0);
      int ng = 0;
      bool any_wall = false;
      for (int i = 0; i < n; ++i) {
        lbm_ctx* c = b->g[i];
        const int ut = ut_t[i];
        if (ut != thermal) continue;
        if (ut && (lbm_get_strip_waves(c) == 2 ? 2 : 1) != waves) continue;
        // arguments of this lattice in its simulated state
        const int sc = c->cur, sT = c->Tcur, sp = c->pcur, sn = c->npart;
        c->cur = st[i].cur;
        c->Tcur = st[i].Tcur;
        c->pcur = st[i].pcur;
        c->npart = st[i].npart;
        LaunchStep L = step_args(c);
        c->cur = sc;
        c->Tcur = sT;
        c->pcur = sp;
        c->npart = sn;
        const bool grav = c->ph.gy != 0.0;
        L.update_T = ut;
        L.want_mass = grav;
        if (grav && c->p.walls) {
          LaunchWall W = wall_args(c, L);
          fill_wall_desc(W, wbuf.data());
          wsig.append(wbuf.data(), wbuf.size());
          wstarts.push_back(wstarts.back() + wall_blocks(c->p.nx));
          L.nwall_in = wall_blocks(c->p.nx);
          any_wall = true;
        } else {
          wstarts.push_back(wstarts.back());  // no wall workgroups for this lattice
          std::memset(wbuf.data(), 0, wbuf.size());
          wsig.append(wbuf.data(), wbuf.size());
        }
        fill_step_desc(L, buf.data());
        sig.append(buf.data(), buf.size());
        starts.push_back(starts.back() + (L.ntx * L.nty + 7) / 8 * 8);
        ++ng;
        // state transition of lbm_step
        st[i].cur ^= 1;
        if (ut) st[i].Tcur ^= 1;
        if (grav) {
          st[i].pcur ^= 1;
          st[i].npart = c->L.nblocks;
        }
        ++st[i].step;
      }
      if (ng == 0) continue;
      sig.append(reinterpret_cast<const char*>(starts.data()), starts.size() * sizeof(int));
      LaunchRec r;
      r.thermal = thermal;
      r.waves = waves;
      r.ngrid = ng;
      r.nblocks = starts.back();
      auto it = seen.find(sig);
      if (it == seen.end()) {
        if (int(tabs.size()) >= kMaxTables) {
          b->err = "schedule needs more distinct launch configurations than the batch buffer holds";
          return LBM_E_UNSUPPORTED;
        }
        it = seen.emplace(sig, int(tabs.size())).first;
        tabs.push_back(sig);
      }
      r.table = it->second;
      if (any_wall) {
        wsig.append(reinterpret_cast<const char*>(wstarts.data()), wstarts.size() * sizeof(int));
        auto wi = wseen.find(wsig);
        if (wi == wseen.end()) {
          if (int(wtabs.size()) >= kMaxTables) {
            b->err = "too many distinct wall-closure configurations";
            return LBM_E_UNSUPPORTED;
          }
          wi = wseen.emplace(wsig, int(wtabs.size())).first;
          wtabs.push_back(wsig);
        }
        r.wall_table = wi->second;
        r.wall_nblocks = wstarts.back();
      }
      recs.push_back(r);
    }
  }
  // --- bring the device tables up to date (host -> device, changed ones only).
  // The launches run on the caller's stream: a table is only overwritten
  // once the work already queued there (which may read it) has finished.
  bool copied = false;
  auto after_user = [&]() -> lbm_status {
    if (copied) return LBM_OK;
    BTRY(b, hipEventRecord(b->join, b->user));
    BTRY(b, hipStreamWaitEvent(b->own, b->join, 0));
    return LBM_OK;
  };
  for (size_t k = 0; k < tabs.size(); ++k) {
    if (k < b->dtab.size() && b->dtab[k] == tabs[k]) continue;
    if (lbm_status q = after_user(); q != LBM_OK) return q;
    const std::string& s = tabs[k];
    const size_t nstart = size_t(recs_ngrid_of(s, b->sdesc)) + 1;
    const size_t db = s.size() - nstart * sizeof(int);
    BTRY(b, hipMemcpyAsync(b->step_tab(int(k)), s.data(), db, hipMemcpyHostToDevice, b->own));
    BTRY(b, hipMemcpyAsync(b->starts(int(k)), s.data() + db, nstart * sizeof(int), hipMemcpyHostToDevice,
                           b->own));
    if (b->dtab.size() <= k) b->dtab.resize(k + 1);
    b->dtab[k] = s;
    copied = true;
  }
  for (size_t k = 0; k < wtabs.size(); ++k) {
    if (k < b->dwtab.size() && b->dwtab[k] == wtabs[k]) continue;
    if (lbm_status q = after_user(); q != LBM_OK) return q;
    const std::string& s = wtabs[k];
    const size_t nstart = size_t(recs_ngrid_of(s, b->wdesc)) + 1;
    const size_t db = s.size() - nstart * sizeof(int);
    BTRY(b, hipMemcpyAsync(b->wall_tab(int(k)), s.data(), db, hipMemcpyHostToDevice, b->own));
    BTRY(b, hipMemcpyAsync(b->wstarts(int(k)), s.data() + db, nstart * sizeof(int), hipMemcpyHostToDevice,
                           b->own));
    if (b->dwtab.size() <= k) b->dwtab.resize(k + 1);
    b->dwtab[k] = s;
    copied = true;
  }
  if (copied) BTRY(b, hipStreamSynchronize(b->own));
  return LBM_OK;
}

static bool same_rec(const LaunchRec& x, const LaunchRec& y) {
  return x.table == y.table && x.wall_table == y.wall_table && x.thermal == y.thermal &&
         x.waves == y.waves && x.ngrid == y.ngrid && x.nblocks == y.nblocks &&
         x.wall_nblocks == y.wall_nblocks;
}

// The graph of m repetitions of the launch pair (x, y), captured on the
// batch's stream on first use and kept until the batch is destroyed.
static lbm_status pair_graph(lbm_batch* b, const LaunchRec& x, const LaunchRec& y, size_t m,
                             hipGraphExec_t* out) {
  const int key_i[] = {x.table, x.wall_table, x.thermal, x.waves, x.ngrid, x.nblocks, x.wall_nblocks,
                       y.table, y.wall_table, y.thermal, y.waves, y.ngrid, y.nblocks, y.wall_nblocks,
                       int(m)};
  const std::string key(reinterpret_cast<const char*>(key_i), sizeof key_i);
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) {
    *out = it->second;
    return LBM_OK;
  }
  hipGraph_t graph;
  hipGraphExec_t exec;
  BTRY(b, hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
  for (size_t k = 0; k < m; ++k) {
    lbm_status s1 = issue(b, x, b->own);
    lbm_status s2 = s1 == LBM_OK ? issue(b, y, b->own) : s1;
    if (s2 != LBM_OK) {
      (void)hipStreamEndCapture(b->own, &graph);
      return s2;
    }
  }
  BTRY(b, hipStreamEndCapture(b->own, &graph));
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  BTRY(b, e);
  b->graphs.emplace(key, exec);
  // move the executable graph to the device now, not at its first launch
  // (done before the graph is launched on the caller's stream)
  BTRY(b, hipGraphUpload(exec, b->own));
  BTRY(b, hipStreamSynchronize(b->own));
  *out = exec;
  return LBM_OK;
}

// Walk the records: runs of a repeated pair go through cached graphs of up
// to kGraphPairs pairs, the rest are launched one by one, on stream st.
// launch = false only makes sure the graphs exist (lbm_batch_prepare).
static lbm_status issue_all(lbm_batch* b, const std::vector<LaunchRec>& recs, int use_graph, bool launch,
                            hipStream_t st) {
  size_t i = 0;
  while (i < recs.size()) {
    size_t reps = 0;
    if (use_graph && i + 3 < recs.size()) {
      while (i + 2 * reps + 3 < recs.size() && same_rec(recs[i + 2 * reps + 2], recs[i]) &&
             same_rec(recs[i + 2 * reps + 3], recs[i + 1]))
        ++reps;
      ++reps;  // the first pair itself
    }
    if (reps >= 2) {
      const size_t m = std::min<size_t>(reps, kGraphPairs);
      hipGraphExec_t exec;
      lbm_status s = pair_graph(b, recs[i], recs[i + 1], m, &exec);
      if (s != LBM_OK) return s;
      const size_t rounds = reps / m;
      if (launch) {
        for (size_t k = 0; k < rounds; ++k) BTRY(b, hipGraphLaunch(exec, st));
        b->graph_launches += int64_t(rounds);
        b->launches += int64_t(rounds * m * 2);
      }
      i += rounds * m * 2;
      continue;
    }
    if (launch) {
      lbm_status s = issue(b, recs[i], st);
      if (s != LBM_OK) return s;
      ++b->launches;
    }
    ++i;
  }
  return LBM_OK;
}

// identity of a run request: the schedule, the graph flag and every
// lattice's host state (a plan depends on nothing else)
static std::string plan_key(const lbm_batch* b, const int64_t* steps, int32_t use_graph) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
  put(&use_graph, sizeof use_graph);
  for (size_t i = 0; i < b->g.size(); ++i) {
    const lbm_ctx* c = b->g[i];
    const int64_t v[] = {steps[i], c->cur, c->Tcur, c->pcur, c->npart, c->step, c->L.ty,
                         lbm_get_strip_waves(c), int64_t(c->generation)};
    put(v, sizeof v);
  }
  return k;
}

lbm_status lbm_batch_prepare(lbm_batch* b, const int64_t* steps, int32_t use_graph) {
  if (!b || !steps) return LBM_E_INVAL;
  std::vector<LaunchRec> recs;
  std::vector<SimState> st;
  b->plan_key.clear();
  lbm_status s = plan_run(b, steps, recs, st);
  if (s != LBM_OK) return s;
  s = issue_all(b, recs, use_graph, false, b->own);
  if (s != LBM_OK) return s;
  BTRY(b, hipStreamSynchronize(b->own));  // uploads done before the timed run
  b->plan_key = plan_key(b, steps, use_graph);
  b->plan_recs.swap(recs);
  b->plan_end.swap(st);
  return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch* b, const int64_t* steps, int32_t use_graph) {
  if (!b || !steps) return LBM_E_INVAL;
  const int n = int(b->g.size());
  std::vector<LaunchRec> recs;
  std::vector<SimState> st;
  lbm_status s = LBM_OK;
  if (!b->plan_key.empty() && b->plan_key == plan_key(b, steps, use_graph)) {
    // prepared for exactly this run: its tables are in device memory and its
    // graphs instantiated (tables are only re-uploaded by a later plan)
    recs.swap(b->plan_recs);
    st.swap(b->plan_end);
  } else {
    s = plan_run(b, steps, recs, st);
    if (s != LBM_OK) return s;
  }
  b->plan_key.clear();
  // the launches go on the caller's stream, ordered after its earlier work
  // and before its later work; the batch's own stream only captures graphs
  // and uploads tables, both finished before this point (a cross-stream
  // event wait here cost 17-25 us of host time before the first launch)
  BTRY(b, hipEventRecord(b->t0, b->user));
  b->launches = 0;
  b->graph_launches = 0;
  s = issue_all(b, recs, use_graph, true, b->user);
  if (s != LBM_OK) return s;
  BTRY(b, hipEventRecord(b->t1, b->user));
  b->timed = true;
  for (int k = 0; k < n; ++k) {
    lbm_ctx* c = b->g[k];
    c->cur = st[k].cur;
    c->Tcur = st[k].Tcur;
    c->pcur = st[k].pcur;
    c->npart = st[k].npart;
    c->step = st[k].step;
    ++c->generation;
  }
  return LBM_OK;
}

lbm_status lbm_batch_last_time(lbm_batch* b, double* ms, int64_t* kernel_launches, int64_t* graph_launches) {
  if (!b || !ms) return LBM_E_INVAL;
  if (!b->timed) return LBM_E_STATE;
  BTRY(b, hipEventSynchronize(b->t1));
  float f = 0.f;
  BTRY(b, hipEventElapsedTime(&f, b->t0, b->t1));
  *ms = f;
  if (kernel_launches) *kernel_launches = b->launches;
  if (graph_launches) *graph_launches = b->graph_launches;
  return LBM_OK;
}

// ------------------------------------------------------------ autotuner
lbm_status lbm_autotune_tile_y(lbm_ctx* c, const int32_t* cand, int32_t n, int32_t steps, int32_t* best_ty,
                               double* best_ms) {
  if (!c || !cand || n < 1 || steps < 1 || !best_ty) return LBM_E_INVAL;
  if (!c->initialized) return fail(c, LBM_E_STATE, "autotune before init");
  double best = 1e300;
  int bt = c->L.ty;
  for (int k = 0; k < n; ++k) {
    if (lbm_set_tile_y(c, cand[k]) != LBM_OK) continue;
    lbm_status s = lbm_step(c, 2);  // warm-up
    if (s != LBM_OK) return s;
    s = lbm_step(c, steps);
    if (s != LBM_OK) return s;
    double ms = 0;
    s = lbm_last_step_time(c, &ms);
    if (s != LBM_OK) return s;
    if (ms < best) {
      best = ms;
      bt = cand[k];
    }
  }
  lbm_status s = lbm_set_tile_y(c, bt);
  if (s != LBM_OK) return s;
  *best_ty = bt;
  if (best_ms) *best_ms = best / steps;
  return lbm_sync(c);
}

lbm_status lbm_tile_candidates(const lbm_ctx* c, int32_t waves, int32_t* out, int32_t cap,
                               int32_t* count) {
  if (!c || !count || waves < 0 || waves > 2 || cap < 0) return LBM_E_INVAL;
  if (waves == 0) waves = lbm_get_strip_waves(c);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, c->base) != hipSuccess) return LBM_E_HIP;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, attr.device) != hipSuccess ||
      cus < 1)
    return LBM_E_HIP;
  constexpr int kSimdsPerCU = 4;
  const int ny = c->p.ny, hi = std::max(ny, 2);
  const long long per_strip = static_cast<long long>(c->L.ntx) * waves;
  std::vector<int32_t> h;
  for (int m = 1; m <= 16; ++m) {
    const long long strips = static_cast<long long>(m) * kSimdsPerCU * cus / per_strip;
    if (strips < 1) continue;
    const int ty = static_cast<int>(std::min<long long>(hi, std::max<long long>(2, (ny + strips - 1) / strips)));
    h.push_back(ty);
  }
  std::sort(h.begin(), h.end());
  h.erase(std::unique(h.begin(), h.end()), h.end());
  for (int k = 0; k < static_cast<int>(h.size()) && k < cap; ++k) out[k] = h[k];
  *count = static_cast<int32_t>(h.size());
  return LBM_OK;
}

}  // extern "C"
