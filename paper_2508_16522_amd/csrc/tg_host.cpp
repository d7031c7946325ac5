// Host side of the C ABI: graph building, compilation into a worker layout,
// launches, reads, batches and the plain comparators.
//
// Compilation follows Algorithm 1 (Compile): the graph's vertices are
// partitioned over workers, every vertex gets a counter of pending in-edges
// and an O(1) list of out-edges.  Three static partitions are offered: the
// default sorts vertices by dependence level and deals them round-robin (a
// graph as wide as the worker count keeps every column on one worker);
// a spread order stretches every graph's levels over one common interval
// first; a list schedule simulates the workers with estimated task costs
// and starts ready vertices longest-remaining-path first.  Every list is
// topologically ordered, which is what makes the executor deadlock-free for
// any ready-window length.
#include "taskgraph.h"
#include "tg_internal.h"
#include "tg_ledger.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <unordered_set>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

using tg::ExecParams;
using tg::GraphEnt;
using tg::ReqDev;
using tg::TaskRec;

namespace {

thread_local std::string g_err;

tg_status fail(tg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

}  // namespace

tg_status tg_set_error(tg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

namespace {

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(TG_EDEVICE, "%s: %s", #x, hipGetErrorString(e_));    \
  } while (0)

// ------------------------------------------------------------ allocation

void* (*g_alloc)(size_t, void*) = nullptr;
void (*g_free)(void*, void*) = nullptr;
void* g_ctx = nullptr;
std::atomic<long> g_live{0};
// host time this thread spent in allocator hooks and in host-device copies
thread_local uint64_t t_hook_ns = 0, t_copy_ns = 0;
// device-built layouts: preparing the graphs' device buffers, and the rest
// of the layout (buffers, tables, kernels) after the blobs were staged
thread_local uint64_t t_setup_ns = 0, t_tables_ns = 0;

uint64_t steady_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void* (*fa)(size_t, void*) = nullptr;
  void (*ff)(void*, void*) = nullptr;
  void* ctx = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      const uint64_t t0 = steady_ns();
      if (ff) ff(p, ctx);
      else (void)hipFree(p);
      t_hook_ns += steady_ns() - t0;
      g_live--;
    }
    p = nullptr;
    bytes = 0;
  }
  tg_status alloc(size_t nbytes) {
    release();
    size_t b = nbytes ? ((nbytes + 255) & ~size_t(255)) : 256;
    fa = g_alloc;
    ff = g_free;
    ctx = g_ctx;
    const uint64_t t0 = steady_ns();
    if (fa) {
      p = fa(b, ctx);
      t_hook_ns += steady_ns() - t0;
      if (!p) return fail(TG_ENOMEM, "device allocation of %zu bytes failed (allocator hook)", b);
    } else {
      hipError_t e = hipMalloc(&p, b);
      t_hook_ns += steady_ns() - t0;
      if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(TG_ENOMEM, "hipMalloc(%zu) failed: %s", b, hipGetErrorString(e));
      }
    }
    bytes = b;
    g_live++;
    return TG_OK;
  }
  template <class T>
  T* as() const { return (T*)p; }
  // Takes over o's memory (o is left empty).
  void take(DevBuf& o) {
    release();
    p = o.p;
    bytes = o.bytes;
    fa = o.fa;
    ff = o.ff;
    ctx = o.ctx;
    o.p = nullptr;
    o.bytes = 0;
  }
};

// Host-to-device copies and memsets here run on the NULL stream (except the
// uploads of the serving builders, on their slot's stream; upload() waits
// for those); for pageable host memory a copy may still be in flight when
// hipMemcpy returns, and the NULL stream is not ordered with the non-blocking
// streams kernels may be launched on.  Every function that prepares device
// data for a launch therefore ends with this fence.
tg_status null_stream_fence() {
  HIPCHK(hipStreamSynchronize(nullptr));
  return TG_OK;
}

// Stream for this thread's uploads; unset, they go to the NULL stream.  The
// serving builder threads set their slot's stream (idle while its batch is
// built) so that their copies do not queue behind one another on the NULL
// stream.  Either way an upload has finished when it returns.
thread_local hipStream_t t_copy_stream = nullptr;

template <class T>
tg_status upload(DevBuf& d, const std::vector<T>& h) {
  tg_status s = d.alloc(h.size() * sizeof(T));
  if (s != TG_OK) return s;
  const uint64_t t0 = steady_ns();
  if (!h.empty()) {
    if (t_copy_stream) {
      HIPCHK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, t_copy_stream));
      HIPCHK(hipStreamSynchronize(t_copy_stream));
    } else {
      HIPCHK(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    }
  }
  t_copy_ns += steady_ns() - t0;
  return TG_OK;
}

uint64_t sm64_host(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------- device info

struct DevInfo {
  int cus = 0;
  int dev = -1;
};

tg_status device_info(DevInfo& di) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t pr;
  HIPCHK(hipGetDeviceProperties(&pr, dev));
  di.cus = pr.multiProcessorCount;
  di.dev = dev;
  return TG_OK;
}

struct Config {
  uint32_t mapping = 1, workers = 0, window = 64, wg_waves = 4, watchdog_ms = 5000, spin_limit = 0, diag = 0;
  uint32_t idle_sleep = 2, notify = 0, schedule = TG_SCHED_LEVEL, gang = 1;
  uint32_t dispatch = TG_DISPATCH_LISTS, tile = 1, shards = 8;
};

Config resolve(const tg_exec_config* c) {
  Config r;
  if (c) {
    if (c->mapping) r.mapping = c->mapping;
    if (c->workers) r.workers = c->workers;
    if (c->window) r.window = c->window;
    if (c->wg_waves) r.wg_waves = c->wg_waves;
    if (c->watchdog_ms) r.watchdog_ms = c->watchdog_ms;
    r.spin_limit = c->spin_limit;
    r.diag = c->diag & 1u;
    r.notify = c->notify & 1u;
    if (c->idle_sleep) r.idle_sleep = c->idle_sleep;
    if (c->schedule) r.schedule = c->schedule;
    if (c->gang) r.gang = c->gang;
    if (c->dispatch) r.dispatch = c->dispatch;
    if (c->tile) r.tile = c->tile;
    if (c->shards) r.shards = c->shards;
  }
  if (r.mapping != TG_MAP_GANG) r.gang = 1;
  return r;
}

tg_status check_config(const Config& c) {
  if (c.mapping != TG_MAP_WAVE && c.mapping != TG_MAP_WORKGROUP && c.mapping != TG_MAP_GANG)
    return fail(TG_EINVAL, "mapping must be 1, 2 or 3");
  if (c.mapping == TG_MAP_GANG && (c.gang < 2 || c.gang > tg::kMaxGang))
    return fail(TG_EINVAL, "gang must be in [2, %u]", tg::kMaxGang);
  if (c.window < 1 || c.window > 64) return fail(TG_EINVAL, "window must be in [1, 64]");
  if (c.idle_sleep < 1 || c.idle_sleep > 64) return fail(TG_EINVAL, "idle_sleep must be in [1, 64]");
  if (c.wg_waves < 1 || c.wg_waves > 16) return fail(TG_EINVAL, "wg_waves must be in [1, 16]");
  if (c.schedule < TG_SCHED_LIST || c.schedule > TG_SCHED_BALANCED) return fail(TG_EINVAL, "schedule must be 1..5");
  if (c.dispatch != TG_DISPATCH_LISTS && c.dispatch != TG_DISPATCH_QUEUE) return fail(TG_EINVAL, "dispatch must be 1 or 2");
  if (c.dispatch == TG_DISPATCH_QUEUE) {
    if (c.mapping == TG_MAP_GANG) return fail(TG_EINVAL, "the ready queue serves wavefront and workgroup workers");
    if (c.tile < 1 || c.tile > 64) return fail(TG_EINVAL, "tile must be in [1, 64]");
    if (c.shards != 1 && c.shards != 2 && c.shards != 4 && c.shards != 8)
      return fail(TG_EINVAL, "shards must be 1, 2, 4 or 8");
  }
  return TG_OK;
}

}  // namespace

// --------------------------------------------------------------- layout

static void ledger_forget(const void* key);

struct Layout {
  Config cfg;
  uint32_t nworkers = 0, grid_blocks = 0, npos = 0, last_started = 0;
  DevBuf rec, pred_addr, succ_pos, indeg, cnt, wbase, gtab, ctrl, execs, wprog, owner, bell, tstamp, wstamp;
  DevBuf q, qctl, qsrc;  // ready-queue dispatch
  uint32_t qwmax = 0;    // most workers claiming from one queue shard
  // layouts built on the device (build_layout_device): the graph tables, the
  // graphs' blobs (staged in pinned host memory, one copy per launch), and
  // per-graph completion (sink counts on the device, flags in host memory)
  DevBuf gsrc, blobs, gdone;
  std::vector<GraphEnt> gtab_host;
  std::vector<tg::GraphSrc> gsrc_host;
  uint32_t* pin = nullptr;
  size_t pin_bytes = 0;
  uint32_t* gflag = nullptr;  // pinned, device-visible
  size_t gflag_n = 0;
  uint32_t gseq = 0;
  std::vector<std::vector<uint32_t>> pos_of;  // per graph: task id -> position
  std::vector<TaskRec> rec_host;               // host copy (rounds can be re-set)
  ExecParams params{};
  double plan_ms = 0, build_ms = 0;  // host time: schedule + records, whole layout incl. upload
  uint64_t signalled = 0;             // edges signalled by a counter atomic per launch
  // residency ledger: kernel variant, co-resident units this layout's launch
  // occupies, the variant's calibrated capacity, device, completion event
  int dev = 0;
  uint64_t variant = 0, units = 0, capacity = 0;
  hipEvent_t ev_done = nullptr;
  Layout() = default;
  Layout(const Layout&) = delete;
  Layout& operator=(const Layout&) = delete;
  ~Layout() {
    ledger_forget(this);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (pin) (void)hipHostFree(pin);
    if (gflag) (void)hipHostFree(gflag);
  }
};

// Process-wide ledger of persistent launches in flight (see tg_ledger.h):
// entries and their completion events, guarded by one lock that is held from
// the decision to the recording of the new launch's completion event.
static std::mutex g_ledger_mu;
static std::vector<tg::Flight> g_flights;
static std::vector<hipEvent_t> g_flight_ev;

static void ledger_forget(const void* key) {
  std::lock_guard<std::mutex> lk(g_ledger_mu);
  for (size_t i = 0; i < g_flights.size(); ++i)
    if (g_flights[i].key == key) {
      g_flights.erase(g_flights.begin() + (ptrdiff_t)i);
      g_flight_ev.erase(g_flight_ev.begin() + (ptrdiff_t)i);
      return;
    }
}

namespace {
struct PlanCache;
}  // namespace

struct tg_graph_s {
  uint32_t mode = 0, n = 0;
  uint64_t space = 0, seed = 0;
  // as built
  std::vector<uint64_t> pred_ptr{0};
  std::vector<uint32_t> preds;
  std::vector<uint32_t> rounds;
  std::vector<uint64_t> req_ptr{0};
  std::vector<tg_region_req> reqs;
  // compiled
  bool finalized = false;
  std::vector<uint64_t> dpred_ptr;  // distinct predecessors (explicit) or inferred (implicit)
  std::vector<uint32_t> dpred;
  std::vector<uint64_t> succ_ptr;
  std::vector<uint32_t> succ;
  std::vector<uint32_t> level;
  // implicit graphs after tg_graph_reduce_edges: the full inferred DAG (what
  // tg_graph_read_dag returns); succ / dpred then hold the reduced edges
  bool reduced = false;
  std::vector<uint64_t> full_succ_ptr;
  std::vector<uint32_t> full_succ;
  // explicit graphs with payload reuse (tg_graph_set_retention): succ holds
  // the data edges plus the anti-dependence edges of reused payload slots,
  // full_succ the data edges alone; topo is the level order the slots were
  // assigned in (a topological order of both edge sets)
  uint32_t retain = TG_KEEP_ALL;
  bool anti = false;
  uint32_t nslots = 0;               // payload slots on the device
  std::vector<uint32_t> slot_of;     // slot of each task (empty: slot v for task v)
  std::vector<uint32_t> slot_last;   // per slot: the task whose payload it holds at the end
  std::vector<uint32_t> topo;
  std::vector<uint32_t> xindeg;      // in-degree over the executed edges (counter reset values)
  std::vector<uint32_t> rw_base;  // implicit: per requirement, ordinal of its first written element
  // The compiled graph in one block of u32 words (built on the host at
  // finalize, uploaded once to `dblob` when the graph first runs): what a
  // launch needs to build task records on the device, and the implicit
  // requirements the records point into (section offsets in words).
  struct BlobOff {
    uint64_t pred_ptr = 0, preds = 0, succ_ptr = 0, succ = 0, indeg = 0, rounds = 0, slot = 0, req_ptr = 0,
             reqs = 0, src = 0, words = 0;
    uint32_t nsrc = 0, nsinks = 0;
    bool has_slot = false;
  } bo;
  std::vector<uint32_t> blob;
  uint64_t blob_gen = 0, dblob_gen = ~0ull;  // host version; version on the device
  DevBuf payload, data, digest, dblob;
  std::unique_ptr<Layout> solo;
  std::shared_ptr<PlanCache> plans;  // schedules of this graph alone, by (workers, schedule)
  // execution state
  bool inflight = false;
  Layout* last_layout = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evk = nullptr;
  double compile_ms = 0, infer_ms = 0, exec_ms = 0, kernel_ms = 0;
  bool has_tuned = false;
  tg_exec_config tuned{};
  // results kept on the host after the device buffers were released
  bool released = false;
  uint64_t dev_gen = 0;  // bumped whenever the device buffers are (re)allocated
  std::vector<uint32_t> host_digest;
  hipStream_t last_stream = nullptr;
  // kernel-time ring: events around the executor kernel of recent launches
  static constexpr uint32_t kRing = 64;
  hipEvent_t rk0[kRing] = {}, rk1[kRing] = {};
  uint64_t launches = 0;
  // comparator hipGraphs: one kernel node per task with one dependency per
  // edge (hg), and the per-task launch sequence captured from a stream (hgc)
  hipGraph_t hg = nullptr, hgc = nullptr;
  hipGraphExec_t hgx = nullptr, hgcx = nullptr;
  uint32_t N() const { return mode == TG_EXPLICIT ? (uint32_t)(pred_ptr.size() - 1) : (uint32_t)(req_ptr.size() - 1); }
};

struct tg_batch_s {
  std::vector<tg_graph> graphs;
  std::vector<uint64_t> gens;  // device-buffer generation of each graph at layout time
  std::unique_ptr<Layout> lay;
  std::shared_ptr<PlanCache> plans;
  bool inflight = false;
  hipStream_t last_stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  static constexpr uint32_t kRing = 64;
  hipEvent_t rk0[kRing] = {}, rk1[kRing] = {};
  uint64_t launches = 0;
};

namespace {

// Largest number of workers of a kernel variant that are proven co-resident
// on the current device.  The occupancy query is only an upper bound (it has
// been observed to over-count on gfx950), so the executor kernel itself is
// launched in probe mode with decreasing blocks-per-CU until every worker
// sees every other worker checked in.  Results are cached per device and
// variant.
struct ResidencyKey {
  int dev;
  uint32_t mapping, wg_waves;
  bool operator<(const ResidencyKey& o) const {
    return std::tie(dev, mapping, wg_waves) < std::tie(o.dev, o.mapping, o.wg_waves);
  }
};
std::mutex g_res_mu;
std::map<ResidencyKey, uint32_t> g_res_cache;

tg_status resident_workers(uint32_t mapping, uint32_t wg_waves, uint32_t* out) {
  DevInfo di;
  tg_status s = device_info(di);
  if (s != TG_OK) return s;
  ResidencyKey key{di.dev, mapping, wg_waves};
  {
    std::lock_guard<std::mutex> lk(g_res_mu);
    auto it = g_res_cache.find(key);
    if (it != g_res_cache.end()) {
      *out = it->second;
      return TG_OK;
    }
  }
  int bpc = tg::exec_blocks_per_cu(mapping, wg_waves);
  if (bpc <= 0) return fail(TG_EDEVICE, "occupancy query failed");
  const uint32_t per_block = mapping == TG_MAP_WAVE ? 4u : 1u;
  // the probe needs the whole device: let launches in flight finish first
  HIPCHK(hipDeviceSynchronize());
  DevBuf ctrl;
  if ((s = ctrl.alloc(sizeof(tg::Ctrl))) != TG_OK) return s;
  uint32_t found = 0;
  for (int b = bpc; b >= 1 && !found; --b) {
    const uint32_t blocks = (uint32_t)b * (uint32_t)di.cus;
    HIPCHK(hipMemset(ctrl.p, 0, sizeof(tg::Ctrl)));
    ExecParams P;
    memset(&P, 0, sizeof(P));
    P.ctrl = ctrl.as<tg::Ctrl>();
    P.nworkers = blocks * per_block;
    P.residency_probe = 1;
    P.watchdog_ticks = 20ull * 100000ull;  // 20 ms
    HIPCHK(tg::launch_exec(P, mapping, wg_waves, blocks, nullptr));
    HIPCHK(hipDeviceSynchronize());
    tg::Ctrl c;
    HIPCHK(hipMemcpy(&c, ctrl.p, sizeof(c), hipMemcpyDeviceToHost));
    if (c.resident == P.nworkers) found = P.nworkers;
  }
  if (!found) return fail(TG_EDEVICE, "no co-resident worker count found");
  std::lock_guard<std::mutex> lk(g_res_mu);
  g_res_cache[key] = found;
  *out = found;
  return TG_OK;
}

// Host part of the layout: everything the kernels read, built on the CPU.
struct HostLayout {
  uint32_t N = 0, nw = 0;
  std::vector<uint32_t> wbase;
  std::vector<TaskRec> rec;
  std::vector<uint64_t> pred_addr;
  std::vector<uint32_t> succ_pos;
  std::vector<uint32_t> indeg;
  std::vector<GraphEnt> gtab;
  std::vector<std::vector<uint32_t>> pos_of;
};

// Estimated cost of a task, in lane-steps of one wavefront: a fixed latency
// term (counter poll, payload hand-off, edge signals) plus the words it
// touches times the mix rounds.  Only the schedule uses it; it is never 0.
uint64_t task_cost(const tg_graph g, uint32_t v) {
  constexpr uint64_t kLatency = 64;
  const uint64_t R = g->rounds[v];
  if (g->mode == TG_EXPLICIT) {
    const uint64_t npred = g->dpred_ptr[v + 1] - g->dpred_ptr[v];
    return kLatency + (uint64_t)g->n / 64 * (R + npred + 1);
  }
  uint64_t ro = 0, rw = 0;
  for (uint64_t i = g->req_ptr[v]; i < g->req_ptr[v + 1]; ++i) {
    const tg_region_req& q = g->reqs[i];
    const uint64_t len = q.hi > q.lo ? q.hi - q.lo : 0;
    (q.priv == TG_RW ? rw : ro) += len;
  }
  return kLatency + (ro + rw * (R + 2)) / 64;
}

// Dependence-level order: all tasks sorted by (level, graph, id) and dealt
// round-robin, so worker w takes entries w, w + nw, ...
void schedule_levels(const std::vector<tg_graph>& gs, uint32_t N, uint32_t nw, std::vector<uint32_t>& wlen,
                     std::vector<uint64_t>& seq) {
  uint32_t maxlevel = 0;
  for (auto g : gs)
    for (uint32_t lv : g->level) maxlevel = std::max(maxlevel, lv);
  std::vector<uint64_t> lstart((size_t)maxlevel + 2, 0);
  for (auto g : gs)
    for (uint32_t lv : g->level) lstart[lv + 1]++;
  for (size_t i = 1; i < lstart.size(); ++i) lstart[i] += lstart[i - 1];
  std::vector<uint64_t> sorted(N);
  for (uint32_t gi = 0; gi < gs.size(); ++gi) {
    const auto& lv = gs[gi]->level;
    for (uint32_t v = 0; v < lv.size(); ++v) sorted[lstart[lv[v]]++] = ((uint64_t)gi << 32) | v;
  }
  wlen.assign(nw, 0);
  for (uint32_t w = 0; w < nw; ++w) wlen[w] = (N > w) ? (N - w + nw - 1) / nw : 0;
  // seq lists worker 0's tasks, then worker 1's, ...
  std::vector<uint64_t> off(nw + 1, 0);
  for (uint32_t w = 0; w < nw; ++w) off[w + 1] = off[w] + wlen[w];
  seq.assign(N, 0);
  for (uint64_t si = 0; si < N; ++si) seq[off[si % nw] + si / nw] = sorted[si];
}

// Spread order: every graph's dependence levels are stretched over the same
// unit interval (task i of the m tasks at level l of an L-level graph gets
// the key (l + (i + 1/2) / m) / L), all tasks are sorted by key and dealt
// round-robin.  Graphs of different depths then advance side by side, and a
// shallow graph's tasks (a dependence-free graph is one level) are spread
// evenly through every worker's list, where the ready window finds them
// whenever the next deep-graph task is not ready yet.  A predecessor's key
// is below its successor's (its level is lower), and ties after
// quantisation keep (graph, id) order, so the sequence is topological.
void schedule_spread(const std::vector<tg_graph>& gs, uint32_t N, uint32_t nw, std::vector<uint32_t>& wlen,
                     std::vector<uint64_t>& seq) {
  const uint64_t Q = std::max<uint64_t>(1024, std::min<uint64_t>(1ull << 24, 2ull * N));
  // key = (l + (i + 1/2) / m) / L = (2 (l m + i) + 1) / (2 m L), kept exact as
  // num / den (both below 2^63 for fewer than 2^32 tasks); its double value
  // only picks the bucket, which is monotone in the exact key
  std::vector<uint64_t> num(N), den(N);
  std::vector<uint32_t> bucket(N);
  std::vector<uint64_t> start(Q + 1, 0);
  uint32_t x = 0;
  for (auto g : gs) {
    const uint32_t n = g->N();
    uint32_t L = 0;
    for (uint32_t lv : g->level) L = std::max(L, lv + 1);
    std::vector<uint32_t> width(L, 0), seen(L, 0);
    for (uint32_t lv : g->level) width[lv]++;
    for (uint32_t v = 0; v < n; ++v, ++x) {
      const uint32_t lv = g->level[v];
      const uint64_t i = seen[lv]++;
      num[x] = 2 * ((uint64_t)lv * width[lv] + i) + 1;
      den[x] = 2 * (uint64_t)width[lv] * L;
      const double k = (lv + (i + 0.5) / width[lv]) / L;
      bucket[x] = (uint32_t)std::min<uint64_t>((uint64_t)(k * (double)Q), Q - 1);
      start[bucket[x] + 1]++;
    }
  }
  for (uint64_t i = 1; i <= Q; ++i) start[i] += start[i - 1];
  std::vector<uint64_t> sorted(N);
  std::vector<uint32_t> idx(N);
  {
    std::vector<uint64_t> fill(start.begin(), start.end() - 1);
    x = 0;
    for (uint32_t gi = 0; gi < gs.size(); ++gi)
      for (uint32_t v = 0; v < gs[gi]->N(); ++v, ++x) {
        sorted[fill[bucket[x]]] = ((uint64_t)gi << 32) | v;
        idx[fill[bucket[x]]++] = x;
      }
  }
  // inside a bucket: by exact key, equal keys (only tasks of different
  // graphs) by (graph, id)
  for (uint64_t q = 0; q < Q; ++q) {
    const uint64_t a = start[q], b = start[q + 1];
    if (b - a < 2) continue;
    std::vector<std::pair<uint32_t, uint64_t>> items;
    for (uint64_t i = a; i < b; ++i) items.emplace_back(idx[i], sorted[i]);
    std::sort(items.begin(), items.end(), [&](const std::pair<uint32_t, uint64_t>& u, const std::pair<uint32_t, uint64_t>& w) {
      const unsigned __int128 l = (unsigned __int128)num[u.first] * den[w.first];
      const unsigned __int128 r = (unsigned __int128)num[w.first] * den[u.first];
      if (l != r) return l < r;
      return u.second < w.second;
    });
    for (uint64_t i = a; i < b; ++i) sorted[i] = items[i - a].second;
  }
  wlen.assign(nw, 0);
  for (uint32_t w = 0; w < nw; ++w) wlen[w] = (N > w) ? (N - w + nw - 1) / nw : 0;
  std::vector<uint64_t> off(nw + 1, 0);
  for (uint32_t w = 0; w < nw; ++w) off[w + 1] = off[w] + wlen[w];
  seq.assign(N, 0);
  for (uint64_t si = 0; si < N; ++si) seq[off[si % nw] + si / nw] = sorted[si];
}

// Column order: task i of level l of a graph goes to worker (o_g + i) mod nw,
// where o_g packs the graphs side by side by their widest level, and every
// worker's list is sorted by the spread key (l + (i + 1/2) / m) / L (exact;
// ties by graph, id).  A graph as wide as its share of the workers keeps each
// column on one worker at every level, and a shallow graph's tasks (a
// dependence-free graph is one level) are spread through every worker's list
// between the deep graphs' tasks.  Keys grow along every edge, so each list
// is topological and the task with the smallest unfinished key is always
// ready at the head of its list.
void schedule_columns(const std::vector<tg_graph>& gs, uint32_t N, uint32_t nw, std::vector<uint32_t>& wlen,
                      std::vector<uint64_t>& seq) {
  std::vector<uint64_t> num(N), den(N);
  std::vector<uint32_t> worker(N);
  uint64_t off = 0;
  uint32_t x = 0;
  for (auto g : gs) {
    uint32_t L = 0;
    for (uint32_t lv : g->level) L = std::max(L, lv + 1);
    std::vector<uint32_t> width(L, 0), seen(L, 0);
    for (uint32_t lv : g->level) width[lv]++;
    uint32_t wmax = 0;
    for (uint32_t w : width) wmax = std::max(wmax, w);
    for (uint32_t v = 0; v < g->N(); ++v, ++x) {
      const uint32_t lv = g->level[v];
      const uint64_t i = seen[lv]++;
      num[x] = 2 * ((uint64_t)lv * width[lv] + i) + 1;
      den[x] = 2 * (uint64_t)width[lv] * L;
      worker[x] = (uint32_t)((off + i) % nw);
    }
    off += wmax;
  }
  wlen.assign(nw, 0);
  for (uint32_t k = 0; k < N; ++k) wlen[worker[k]]++;
  std::vector<uint64_t> start(nw + 1, 0);
  for (uint32_t w = 0; w < nw; ++w) start[w + 1] = start[w] + wlen[w];
  std::vector<uint32_t> idx(N);
  {
    std::vector<uint64_t> fill(start.begin(), start.end() - 1);
    for (uint32_t k = 0; k < N; ++k) idx[fill[worker[k]]++] = k;
  }
  // graph and id of global index k
  std::vector<uint64_t> key_of(N);
  x = 0;
  for (uint32_t gi = 0; gi < gs.size(); ++gi)
    for (uint32_t v = 0; v < gs[gi]->N(); ++v, ++x) key_of[x] = ((uint64_t)gi << 32) | v;
  seq.assign(N, 0);
  for (uint32_t w = 0; w < nw; ++w) {
    auto b = idx.begin() + start[w], e = idx.begin() + start[w + 1];
    std::sort(b, e, [&](uint32_t u, uint32_t v) {
      const unsigned __int128 l = (unsigned __int128)num[u] * den[v];
      const unsigned __int128 r = (unsigned __int128)num[v] * den[u];
      return l != r ? l < r : u < v;
    });
    for (uint64_t k = start[w]; k < start[w + 1]; ++k) seq[k] = key_of[idx[k]];
  }
}

// Balanced level order: tasks in (dependence level, graph, id) order, each
// given to the worker with the least estimated work so far (costs as for the
// list schedule).  Every list is a subsequence of the level order, so it is
// topological; the workers' total work stays even when task costs differ by
// orders of magnitude (graphs of very different payloads and mix rounds).
void schedule_balanced(const std::vector<tg_graph>& gs, uint32_t N, uint32_t nw, std::vector<uint32_t>& wlen,
                       std::vector<uint64_t>& seq) {
  uint32_t maxlevel = 0;
  for (auto g : gs)
    for (uint32_t lv : g->level) maxlevel = std::max(maxlevel, lv);
  std::vector<uint64_t> lstart((size_t)maxlevel + 2, 0);
  for (auto g : gs)
    for (uint32_t lv : g->level) lstart[lv + 1]++;
  for (size_t i = 1; i < lstart.size(); ++i) lstart[i] += lstart[i - 1];
  std::vector<uint64_t> sorted(N);
  for (uint32_t gi = 0; gi < gs.size(); ++gi) {
    const auto& lv = gs[gi]->level;
    for (uint32_t v = 0; v < lv.size(); ++v) sorted[lstart[lv[v]]++] = ((uint64_t)gi << 32) | v;
  }
  typedef std::pair<uint64_t, uint32_t> Load;  // (work so far, worker)
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (uint32_t w = 0; w < nw; ++w) heap.push(Load(0, w));
  std::vector<uint32_t> owner(N);
  wlen.assign(nw, 0);
  for (uint64_t si = 0; si < N; ++si) {
    Load l = heap.top();
    heap.pop();
    owner[si] = l.second;
    wlen[l.second]++;
    l.first += task_cost(gs[sorted[si] >> 32], (uint32_t)sorted[si]);
    heap.push(l);
  }
  std::vector<uint64_t> off(nw + 1, 0);
  for (uint32_t w = 0; w < nw; ++w) off[w + 1] = off[w] + wlen[w];
  seq.assign(N, 0);
  for (uint64_t si = 0; si < N; ++si) seq[off[owner[si]]++] = sorted[si];
}

// List schedule: simulate nw identical workers.  Whenever workers are free,
// the ready tasks with the longest remaining path (sum of estimated costs to
// a sink) start on them, in the order the workers became free; a task's
// successors become ready when its simulated run ends.  Ready tasks are kept
// in a bucket queue over the quantised path length (FIFO inside a bucket),
// busy workers in a heap of finish times.  Each worker's list is its tasks in
// simulated start order; since costs are positive, a task starts strictly
// after each of its predecessors, so the lists are topologically ordered.
tg_status schedule_list(const std::vector<tg_graph>& gs, uint32_t N, uint32_t nw, std::vector<uint32_t>& wlen,
                        std::vector<uint64_t>& seq) {
  const uint32_t G = (uint32_t)gs.size();
  std::vector<uint32_t> gbase(G + 1, 0);
  for (uint32_t gi = 0; gi < G; ++gi) gbase[gi + 1] = gbase[gi] + gs[gi]->N();
  std::vector<uint32_t> gof(N);
  for (uint32_t gi = 0; gi < G; ++gi)
    for (uint32_t v = 0; v < gs[gi]->N(); ++v) gof[gbase[gi] + v] = gi;
  // costs and longest remaining paths (ids are a topological order)
  std::vector<uint64_t> cost(N), path(N);
  uint64_t pmax = 1;
  for (uint32_t gi = 0; gi < G; ++gi) {
    const tg_graph g = gs[gi];
    for (uint32_t v = g->N(); v-- > 0;) {
      const uint32_t x = gbase[gi] + v;
      cost[x] = task_cost(g, v);
      uint64_t m = 0;
      for (uint64_t j = g->succ_ptr[v]; j < g->succ_ptr[v + 1]; ++j) m = std::max(m, path[gbase[gi] + g->succ[j]]);
      path[x] = cost[x] + m;
      pmax = std::max(pmax, path[x]);
    }
  }
  // bucket queue: higher bucket = longer path
  constexpr uint32_t kBuckets = 1u << 16;
  std::vector<uint32_t> head(kBuckets, 0xFFFFFFFFu), tail(kBuckets, 0xFFFFFFFFu), next(N, 0xFFFFFFFFu);
  std::vector<uint64_t> nonempty(kBuckets / 64, 0);
  auto bucket_of = [&](uint32_t x) {
    return (uint32_t)(((unsigned __int128)path[x] * (kBuckets - 1)) / pmax);
  };
  auto push = [&](uint32_t x) {
    const uint32_t b = bucket_of(x);
    if (head[b] == 0xFFFFFFFFu) {
      head[b] = x;
      nonempty[b >> 6] |= 1ull << (b & 63);
    } else {
      next[tail[b]] = x;
    }
    tail[b] = x;
    next[x] = 0xFFFFFFFFu;
  };
  int64_t top_word = kBuckets / 64 - 1;
  auto pop = [&]() -> uint32_t {  // highest non-empty bucket, or none
    for (int64_t wi = top_word; wi >= 0; --wi) {
      if (!nonempty[wi]) continue;
      top_word = wi;
      const uint32_t b = (uint32_t)wi * 64 + (63 - __builtin_clzll(nonempty[wi]));
      const uint32_t x = head[b];
      head[b] = next[x];
      if (head[b] == 0xFFFFFFFFu) {
        tail[b] = 0xFFFFFFFFu;
        nonempty[wi] &= ~(1ull << (b & 63));
      }
      return x;
    }
    top_word = 0;
    return 0xFFFFFFFFu;
  };
  std::vector<uint32_t> pend(N);
  for (uint32_t gi = 0; gi < G; ++gi) {
    const tg_graph g = gs[gi];
    for (uint32_t v = 0; v < g->N(); ++v) {
      pend[gbase[gi] + v] = g->xindeg[v];
      if (pend[gbase[gi] + v] == 0) push(gbase[gi] + v);
    }
  }
  auto raise_top = [&](uint32_t x) { top_word = std::max<int64_t>(top_word, bucket_of(x) >> 6); };
  // free workers in the order they became free; busy ones by finish time
  std::vector<uint32_t> freeq(nw);
  for (uint32_t w = 0; w < nw; ++w) freeq[w] = w;
  size_t fq_head = 0;
  typedef std::pair<uint64_t, uint32_t> Busy;  // (finish time, worker)
  std::priority_queue<Busy, std::vector<Busy>, std::greater<Busy>> busy;
  std::vector<uint32_t> running(nw, 0xFFFFFFFFu);
  std::vector<uint32_t> owner(N), order_in(N);
  wlen.assign(nw, 0);
  uint64_t now = 0, started = 0;
  while (started < N) {
    while (fq_head < freeq.size()) {
      const uint32_t x = pop();
      if (x == 0xFFFFFFFFu) break;
      const uint32_t w = freeq[fq_head++];
      owner[x] = w;
      order_in[x] = wlen[w]++;
      running[w] = x;
      busy.push(Busy(now + cost[x], w));
      ++started;
    }
    if (fq_head > nw) {  // drop the consumed prefix of the free queue
      freeq.erase(freeq.begin(), freeq.begin() + (ptrdiff_t)fq_head);
      fq_head = 0;
    }
    if (busy.empty()) break;  // nothing runs and nothing is ready: a cycle
    now = busy.top().first;
    while (!busy.empty() && busy.top().first == now) {
      const uint32_t w = busy.top().second;
      busy.pop();
      const uint32_t x = running[w];
      running[w] = 0xFFFFFFFFu;
      freeq.push_back(w);
      const uint32_t gi = gof[x];
      const tg_graph g = gs[gi];
      const uint32_t v = x - gbase[gi];
      for (uint64_t j = g->succ_ptr[v]; j < g->succ_ptr[v + 1]; ++j) {
        const uint32_t y = gbase[gi] + g->succ[j];
        if (--pend[y] == 0) {
          push(y);
          raise_top(y);
        }
      }
    }
  }
  if (started < N) return fail(TG_EINVAL, "dependence cycle: %llu of %u tasks schedulable",
                               (unsigned long long)started, N);
  std::vector<uint64_t> off(nw + 1, 0);
  for (uint32_t w = 0; w < nw; ++w) off[w + 1] = off[w] + wlen[w];
  seq.assign(N, 0);
  for (uint32_t x = 0; x < N; ++x) {
    const uint32_t gi = gof[x];
    seq[off[owner[x]] + order_in[x]] = ((uint64_t)gi << 32) | (x - gbase[gi]);
  }
  return TG_OK;
}

// Schedule a set of finalised graphs onto nw workers (list schedule or
// dependence-level order) and store each worker's tasks contiguously in the
// order it is to run them.
// A schedule: per-worker list lengths and, worker by worker, the tasks of
// each list in order as (graph << 32) | id.
uint64_t req_addr(tg_graph g, uint32_t v);

// Per-graph constants of the graph table.
void graph_entry(tg_graph g, GraphEnt& e) {
  memset(&e, 0, sizeof(e));
  e.key1 = sm64_host(g->seed ^ (1ull << 32));
  e.key2 = sm64_host(g->seed ^ (2ull << 32));
  e.digest = g->digest.as<uint32_t>();
  e.data = g->data.as<uint32_t>();
  e.n = g->n;
  e.mode = g->mode;
  e.nsinks = g->bo.nsinks;
}

struct Plan {
  std::vector<uint32_t> wlen;
  std::vector<uint64_t> seq;
};

tg_status plan_layout(const std::vector<tg_graph>& gs, uint64_t nw_req, uint32_t schedule, HostLayout& H,
                      const Plan* reuse = nullptr, Plan* keep = nullptr) {
  uint64_t ntot = 0, npred_tot = 0, nsucc_tot = 0, nreq_tot = 0;
  for (auto g : gs) {
    ntot += g->N();
    npred_tot += g->mode == TG_EXPLICIT ? g->dpred.size() : 0;
    nsucc_tot += g->succ.size();
    nreq_tot += g->mode == TG_IMPLICIT ? g->reqs.size() : 0;
  }
  if (ntot >= 0xFFFFFFFFull || npred_tot >= 0xFFFFFFFFull || nsucc_tot >= 0xFFFFFFFFull || nreq_tot >= 0xFFFFFFFFull)
    return fail(TG_EINVAL, "layout too large: %llu tasks, %llu edges", (unsigned long long)ntot,
                (unsigned long long)nsucc_tot);
  if (schedule < TG_SCHED_LIST || schedule > TG_SCHED_BALANCED) return fail(TG_EINVAL, "schedule must be 1..5");
  const uint32_t N = (uint32_t)ntot;
  uint64_t nw = nw_req;
  if (nw > N) nw = N ? N : 1;
  if (nw == 0) nw = 1;
  H.N = N;
  H.nw = (uint32_t)nw;
  std::vector<uint32_t> wlen;
  std::vector<uint64_t> at_pos;  // (graph << 32) | id, by position
  if (reuse && reuse->wlen.size() == nw && reuse->seq.size() == N) {
    wlen = reuse->wlen;
    at_pos = reuse->seq;
  } else if (schedule == TG_SCHED_LIST) {
    tg_status st = schedule_list(gs, N, (uint32_t)nw, wlen, at_pos);
    if (st != TG_OK) return st;
  } else if (schedule == TG_SCHED_LEVEL) {
    schedule_levels(gs, N, (uint32_t)nw, wlen, at_pos);
  } else if (schedule == TG_SCHED_SPREAD) {
    schedule_spread(gs, N, (uint32_t)nw, wlen, at_pos);
  } else if (schedule == TG_SCHED_COLUMN) {
    schedule_columns(gs, N, (uint32_t)nw, wlen, at_pos);
  } else {
    schedule_balanced(gs, N, (uint32_t)nw, wlen, at_pos);
  }
  if (keep) {
    keep->wlen = wlen;
    keep->seq = at_pos;
  }
  H.wbase.assign((size_t)nw + 1, 0);
  for (uint64_t w = 0; w < nw; ++w) H.wbase[w + 1] = H.wbase[w] + wlen[w];
  H.pos_of.assign(gs.size(), {});
  for (uint32_t gi = 0; gi < gs.size(); ++gi) H.pos_of[gi].assign(gs[gi]->N(), 0);
  for (uint32_t pos = 0; pos < N; ++pos) H.pos_of[at_pos[pos] >> 32][(uint32_t)at_pos[pos]] = pos;
  // records by position, edge arrays (every element is written below)
  H.rec.resize(N);
  H.pred_addr.resize(npred_tot);
  H.succ_pos.resize(nsucc_tot);
  H.indeg.resize(N);
  // records in graph order (each graph's arrays are read sequentially); a
  // record is stored at its task's position, and its predecessor and
  // successor lists are slices of pred_addr / succ_pos in graph order.
  // Large layouts split the tasks over a few threads.
  std::vector<uint64_t> gfirst(gs.size() + 1, 0), pbase(gs.size(), 0), sbase(gs.size(), 0);
  {
    uint64_t pb = 0, sb = 0;
    for (uint32_t gi = 0; gi < gs.size(); ++gi) {
      gfirst[gi + 1] = gfirst[gi] + gs[gi]->N();
      pbase[gi] = pb;
      sbase[gi] = sb;
      if (gs[gi]->mode == TG_EXPLICIT) pb += gs[gi]->dpred.size();
      sb += gs[gi]->succ.size();
    }
  }
  auto build_range = [&](uint64_t lo, uint64_t hi) {  // global task indices [lo, hi)
    uint32_t gi = (uint32_t)(std::upper_bound(gfirst.begin(), gfirst.end(), lo) - gfirst.begin()) - 1;
    for (uint64_t x = lo; x < hi; ++gi) {
      const tg_graph g = gs[gi];
      const std::vector<uint32_t>& pos = H.pos_of[gi];
      const bool expl = g->mode == TG_EXPLICIT;
      const uint64_t base = expl ? (uint64_t)g->payload.p : 0, wbytes = (uint64_t)g->n * 4ull;
      const uint64_t pb = pbase[gi], sb = sbase[gi];
      const uint32_t vend = (uint32_t)(std::min(hi, gfirst[gi + 1]) - gfirst[gi]);
      for (uint32_t v = (uint32_t)(x - gfirst[gi]); v < vend; ++v, ++x) {
        TaskRec r;
        memset(&r, 0, sizeof(r));
        r.tid = v;
        r.graph = gi;
        r.rounds = g->rounds[v];
        const uint64_t d0 = g->dpred_ptr[v], d1 = g->dpred_ptr[v + 1];
        r.npred = (uint32_t)(d1 - d0);
        if (expl) {
          const bool slots = !g->slot_of.empty();
          r.out = base + (uint64_t)(slots ? g->slot_of[v] : v) * wbytes;
          r.pred_beg = (uint32_t)(pb + d0);
          for (uint64_t j = d0; j < d1; ++j) {
            const uint32_t p = g->dpred[j];
            const uint64_t addr = base + (uint64_t)(slots ? g->slot_of[p] : p) * wbytes;
            if (j - d0 < tg::kInPred) r.pred[j - d0] = addr;
            H.pred_addr[pb + j] = addr;
          }
        } else {
          r.out = req_addr(g, v);
          r.nreq = (uint32_t)(g->req_ptr[v + 1] - g->req_ptr[v]);
        }
        const uint64_t s0 = g->succ_ptr[v], s1 = g->succ_ptr[v + 1];
        r.succ_beg = (uint32_t)(sb + s0);
        r.nsucc = (uint32_t)(s1 - s0);
        for (uint64_t j = s0; j < s1; ++j) {
          const uint32_t sp = pos[g->succ[j]];
          if (j - s0 < tg::kInSucc) r.succ[j - s0] = sp;
          H.succ_pos[sb + j] = sp;
        }
        H.rec[pos[v]] = r;
        H.indeg[pos[v]] = g->xindeg[v];
      }
    }
  };
  // records are written in position order (scattered): worth threads from a
  // few thousand tasks per thread (serving batches are ~10^5 tasks)
  const uint32_t nthreads = N >= (1u << 14) ? std::max(1u, std::min(8u, std::thread::hardware_concurrency())) : 1u;
  if (nthreads <= 1) {
    build_range(0, N);
  } else {
    std::vector<std::thread> pool;
    for (uint32_t t = 0; t < nthreads; ++t)
      pool.emplace_back(build_range, (uint64_t)N * t / nthreads, (uint64_t)N * (t + 1) / nthreads);
    for (auto& th : pool) th.join();
  }
  H.gtab.assign(gs.size(), GraphEnt());
  for (uint32_t gi = 0; gi < gs.size(); ++gi) graph_entry(gs[gi], H.gtab[gi]);
  return TG_OK;
}

// List dispatch: an edge from a list entry to the next entry of the same
// worker's list needs no counter.  The worker finishes its tasks one after
// another, so the earlier task is done before the later one is taken; the
// edge is moved past the end of the earlier task's successors (not
// signalled) and the later task's counter starts one lower, with kAfterPrev
// set (the ready scan then also waits for the entry before it to be taken).
// A dependence chain kept on one worker (a Task Bench column) thus costs no
// atomic and no counter round trip per task.
void elide_list_edges(HostLayout& H) {
  for (uint32_t w = 0; w < H.nw; ++w)
    for (uint32_t p = H.wbase[w] + 1; p < H.wbase[w + 1]; ++p) {
      TaskRec& r = H.rec[p - 1];
      uint32_t* list = H.succ_pos.data() + r.succ_beg;
      for (uint32_t j = 0; j < r.nsucc; ++j)
        if (list[j] == p) {
          std::swap(list[j], list[r.nsucc - 1]);
          r.nsucc--;
          for (uint32_t k = 0; k < tg::kInSucc && k < r.nsucc + 1; ++k) r.succ[k] = list[k];
          H.indeg[p] = (H.indeg[p] - 1u) | tg::kAfterPrev;
          break;
        }
    }
}

// Most workers that claim tickets from one queue shard: a worker claims from
// shard (workgroup index mod 8) mod shards, as the kernels do; wavefront
// workers sit four to a workgroup.
uint32_t queue_workers_per_shard(const Config& cfg, uint32_t nw, uint32_t shards) {
  std::vector<uint32_t> per(shards, 0);
  for (uint32_t w = 0; w < nw; ++w) {
    const uint32_t block = cfg.mapping == TG_MAP_WAVE ? w / 4 : w;
    per[(block & 7u) & (shards - 1u)]++;
  }
  return *std::max_element(per.begin(), per.end());
}

// Shards a launch of nw workers uses: every shard needs a workgroup that
// claims from it (a claimed ticket is only ever run by its claimer, so tasks
// pushed into a shard without workers would never run), so at most as many
// shards as workgroups, rounded down to a power of two.
uint32_t queue_shards(const Config& cfg, uint32_t nw) {
  const uint32_t blocks = cfg.mapping == TG_MAP_WAVE ? (nw + 3) / 4 : nw;
  uint32_t s = cfg.shards;
  while (s > 1 && s > blocks) s >>= 1;
  return s;
}

tg_status ensure_device(tg_graph g, bool upload_blob = true);
tg_status ensure_events(tg_graph g);

// Schedule and upload the layout of a set of finalised graphs.
// Schedules already computed for a set of graphs, by (workers, schedule):
// launch shapes with the same worker count share one, so an autotuner pass
// schedules only new (worker count, schedule) pairs; task records are always
// rebuilt, so they carry the graphs' current mix rounds.
struct PlanCache {
  static constexpr uint64_t kMaxTasks = 1ull << 25;  // larger schedules are not kept
  static constexpr size_t kMaxEntries = 16;
  std::map<std::pair<uint32_t, uint32_t>, std::shared_ptr<const Plan>> m;
};

// keep_host: keep the host copy of the task records in the layout (needed
// to re-set mix rounds later).  Without it the records are built in a
// per-thread host layout whose buffers are reused from call to call.
tg_status build_layout(const std::vector<tg_graph>& gs, const Config& cfg, std::unique_ptr<Layout>& out,
                       PlanCache* cache = nullptr, bool keep_host = true) {
  const auto t_build = std::chrono::steady_clock::now();
  tg_status s = check_config(cfg);
  if (s != TG_OK) return s;
  for (auto g : gs)
    if ((s = ensure_device(g)) != TG_OK) return s;
  uint32_t cap32 = 0;
  // a gang's workgroups are the workgroup executor's (same bounds and
  // occupancy attributes), so its residency is that count over the gang size
  const uint32_t res_mapping = cfg.mapping == TG_MAP_GANG ? (uint32_t)TG_MAP_WORKGROUP : cfg.mapping;
  if ((s = resident_workers(res_mapping, cfg.wg_waves, &cap32)) != TG_OK) return s;
  const uint64_t cap_workers = cap32 / cfg.gang;
  if (cap_workers == 0) return fail(TG_EINVAL, "gang of %u workgroups of %u waves does not fit", cfg.gang, cfg.wg_waves);
  uint64_t nw = cfg.workers ? cfg.workers : cap_workers;
  if (nw > cap_workers) nw = cap_workers;  // every worker must be co-resident
  static thread_local HostLayout tl_host;
  HostLayout local;
  HostLayout& H = keep_host ? local : tl_host;
  const auto t_plan = std::chrono::steady_clock::now();
  const std::pair<uint32_t, uint32_t> key((uint32_t)nw, cfg.schedule);
  const Plan* reuse = nullptr;
  if (cache) {
    auto hit = cache->m.find(key);
    if (hit != cache->m.end()) reuse = hit->second.get();
  }
  uint64_t ntasks = 0;
  for (auto g : gs) ntasks += g->N();
  const bool keep = cache && !reuse && ntasks <= PlanCache::kMaxTasks && cache->m.size() < PlanCache::kMaxEntries;
  auto kept = keep ? std::make_shared<Plan>() : nullptr;
  if ((s = plan_layout(gs, nw, cfg.schedule, H, reuse, kept.get())) != TG_OK) return s;
  // A worker's list order replaces the edges between its consecutive entries
  // only where one team runs the whole task; the members of a gang finish
  // their shares independently, so there every edge is counted once per
  // member and a counter starts at in-degree x gang size.
  if (cfg.dispatch == TG_DISPATCH_LISTS && cfg.mapping != TG_MAP_GANG) elide_list_edges(H);
  if (cfg.mapping == TG_MAP_GANG)
    for (uint32_t& c : H.indeg) {
      if (c > tg::kPendingMask / cfg.gang)
        return fail(TG_EINVAL, "in-degree %u times a gang of %u exceeds the counter range", c, cfg.gang);
      c *= cfg.gang;
    }
  uint64_t signalled = 0;
  for (const TaskRec& r : H.rec) signalled += r.nsucc;
  if (keep) cache->m[key] = kept;
  const double plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_plan).count();
  auto L = std::make_unique<Layout>();
  L->cfg = cfg;
  L->signalled = signalled;
  L->npos = H.N;
  L->nworkers = H.nw;
  L->grid_blocks = cfg.mapping == TG_MAP_WAVE ? (H.nw + 3) / 4 : H.nw * cfg.gang;
  {
    DevInfo di;
    if ((s = device_info(di)) != TG_OK) return s;
    L->dev = di.dev;
    L->variant = (cfg.mapping == TG_MAP_WAVE ? tg::flight_variant(TG_MAP_WAVE, 1, 1)
                                             : tg::flight_variant(cfg.mapping, cfg.wg_waves, cfg.gang)) |
                 ((uint64_t)cfg.dispatch << 60);
    L->units = (uint64_t)H.nw * cfg.gang;  // wavefronts, or workgroups
    L->capacity = cap32;
    HIPCHK(hipEventCreateWithFlags(&L->ev_done, hipEventDisableTiming));
  }
  L->pos_of = std::move(H.pos_of);
  const uint32_t N = H.N;
  // queue dispatch: the sources (pushed at reset) and the number of sinks
  // (the launch ends when all have run)
  std::vector<uint32_t> src;
  uint32_t sinks = 0;
  if (cfg.dispatch == TG_DISPATCH_QUEUE)
    for (uint32_t p = 0; p < N; ++p) {
      if (H.indeg[p] == 0) src.push_back(p);
      if (H.rec[p].nsucc == 0) ++sinks;
    }
  if ((s = upload(L->rec, H.rec)) != TG_OK) return s;
  if (keep_host) L->rec_host = std::move(H.rec);
  if ((s = upload(L->pred_addr, H.pred_addr)) != TG_OK) return s;
  if ((s = upload(L->succ_pos, H.succ_pos)) != TG_OK) return s;
  if ((s = upload(L->indeg, H.indeg)) != TG_OK) return s;
  if ((s = L->cnt.alloc((size_t)N * 4)) != TG_OK) return s;
  if ((s = upload(L->wbase, H.wbase)) != TG_OK) return s;
  if ((s = upload(L->gtab, H.gtab)) != TG_OK) return s;
  if ((s = L->ctrl.alloc(sizeof(tg::Ctrl))) != TG_OK) return s;
  HIPCHK(hipMemset(L->ctrl.p, 0, sizeof(tg::Ctrl)));
  {
    std::vector<uint32_t> own(N);
    for (uint32_t w = 0; w < H.nw; ++w)
      for (uint32_t p = H.wbase[w]; p < H.wbase[w + 1]; ++p) own[p] = w;
    if ((s = upload(L->owner, own)) != TG_OK) return s;
  }
  if ((s = L->bell.alloc((size_t)H.nw * tg::kBellStride * 4)) != TG_OK) return s;
  HIPCHK(hipMemset(L->bell.p, 0, (size_t)H.nw * tg::kBellStride * 4));
  ExecParams& P = L->params;
  P.rec = L->rec.as<TaskRec>();
  P.pred_addr = L->pred_addr.as<uint64_t>();
  P.succ_pos = L->succ_pos.as<uint32_t>();
  P.indeg = L->indeg.as<uint32_t>();
  P.cnt = L->cnt.as<uint32_t>();
  P.wbase = L->wbase.as<uint32_t>();
  P.gtab = L->gtab.as<GraphEnt>();
  P.ctrl = L->ctrl.as<tg::Ctrl>();
  P.owner = L->owner.as<uint32_t>();
  P.bell = L->bell.as<uint32_t>();
  P.gang = cfg.gang;
  P.npos = N;
  P.nworkers = L->nworkers;
  P.window = cfg.window;
  P.spin_limit = cfg.spin_limit;
  P.watchdog_ticks = (uint64_t)cfg.watchdog_ms * 100000ull;
  if (cfg.dispatch == TG_DISPATCH_QUEUE) {
    // Each shard has a ticket slot for every task (each task is pushed once,
    // into one shard) plus the exit sentinels of its workers: tile x (workers
    // claiming from it + 1), sized for the largest tile so that a launch may
    // choose any tile.  All slots start empty; the sources are pushed at reset.
    const uint32_t shards = queue_shards(cfg, H.nw);
    L->qwmax = queue_workers_per_shard(cfg, H.nw, shards);
    const uint64_t cap = (uint64_t)N + 64ull * (L->qwmax + 1);
    if (cap >= 0xFFFFFFF0ull) return fail(TG_EINVAL, "queue of %llu slots per shard is too large", (unsigned long long)cap);
    if ((s = L->q.alloc((size_t)shards * cap * 4)) != TG_OK) return s;
    HIPCHK(hipMemset(L->q.p, 0xFF, (size_t)shards * cap * 4));
    const size_t ctl_bytes = (size_t)(2 * shards + 1) * tg::kQLine * 4;
    if ((s = L->qctl.alloc(ctl_bytes)) != TG_OK) return s;
    HIPCHK(hipMemset(L->qctl.p, 0, ctl_bytes));
    if ((s = upload(L->qsrc, src)) != TG_OK) return s;
    P.q = L->q.as<uint32_t>();
    P.qctl = L->qctl.as<uint32_t>();
    P.qsrc = L->qsrc.as<uint32_t>();
    P.nsrc = (uint32_t)src.size();
    P.nsinks = sinks;
    P.qshards = shards;
    P.qcap = (uint32_t)cap;
    P.qtile = cfg.tile;
    P.qsent = cfg.tile * (L->qwmax + 1);
  }
  if ((s = null_stream_fence()) != TG_OK) return s;
  L->plan_ms = plan_ms;
  L->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_build).count();
  out = std::move(L);
  return TG_OK;
}

// Grows a reusable device buffer to at least `bytes` (by half again, so a
// serving slot reallocates rarely); returns true in *grown when it did.
tg_status grow(DevBuf& b, size_t bytes, bool* grown = nullptr) {
  if (grown) *grown = false;
  if (b.p && b.bytes >= bytes) return TG_OK;
  if (grown) *grown = true;
  return b.alloc(std::max(bytes, b.bytes + b.bytes / 2));
}

// A ready-queue layout whose task records are built on the device from the
// graphs' compiled blobs (k_build_records), for launches that cannot afford
// host planning (serving): the host work is one table entry per graph.
// Positions follow graph order, task ids ascending.  L is reused from launch
// to launch on one stream: its buffers only grow, and the queue slots the
// previous launch filled are emptied first.  Every step runs on `st`.
// Pinned host memory of at least `bytes`, kept and grown (by half again);
// `coherent` asks for fine-grained memory that device stores reach while a
// kernel runs.
tg_status grow_pinned(uint32_t*& p, size_t& have, size_t bytes, bool coherent = false) {
  if (p && have >= bytes) return TG_OK;
  const size_t want = std::max(bytes, have + have / 2);
  if (p) (void)hipHostFree(p);
  p = nullptr;
  have = 0;
  HIPCHK(hipHostMalloc((void**)&p, want, coherent ? (hipHostMallocCoherent | hipHostMallocMapped) : hipHostMallocDefault));
  have = want;
  return TG_OK;
}

tg_status build_layout_device(const std::vector<tg_graph>& gs, const Config& cfg, Layout& L, hipStream_t st,
                              bool report) {
  const auto t_build = std::chrono::steady_clock::now();
  tg_status s = check_config(cfg);
  if (s != TG_OK) return s;
  if (cfg.dispatch != TG_DISPATCH_QUEUE || cfg.mapping == TG_MAP_GANG)
    return fail(TG_EINVAL, "device-built layouts use the ready queue with wavefront or workgroup workers");
  const uint64_t t_setup0 = steady_ns();
  {
    // the graphs' buffers are cleared and their blobs uploaded on `st` too
    const hipStream_t prev = t_copy_stream;
    t_copy_stream = st;
    for (auto g : gs)
      if ((s = ensure_device(g, false)) != TG_OK) break;
    t_copy_stream = prev;
    if (s != TG_OK) return s;
  }
  // the graphs' blobs, packed one after the other (256-byte aligned) into
  // the pinned staging buffer and copied to the device arena in one go; the
  // staging buffer is free again once this layout's previous launch, which
  // is ordered after its copy, has finished
  std::vector<uint64_t> boff(gs.size(), 0);
  uint64_t bwords = 0;
  for (size_t gi = 0; gi < gs.size(); ++gi) {
    boff[gi] = bwords;
    bwords += (gs[gi]->blob.size() + 63) & ~63ull;
  }
  if ((s = grow_pinned(L.pin, L.pin_bytes, std::max<uint64_t>(bwords, 64) * 4)) != TG_OK) return s;
  if ((s = grow(L.blobs, std::max<uint64_t>(bwords, 64) * 4)) != TG_OK) return s;
  {
    // large batches stage on several threads (the blobs are read from
    // memory the cache no longer holds)
    auto stage = [&](size_t g0, size_t g1) {
      for (size_t gi = g0; gi < g1; ++gi)
        if (!gs[gi]->blob.empty()) memcpy(L.pin + boff[gi], gs[gi]->blob.data(), gs[gi]->blob.size() * 4);
    };
    const size_t nth = bwords * 4 >= (8u << 20) ? std::min<size_t>(gs.size(), 6) : 1;
    if (nth <= 1) {
      stage(0, gs.size());
    } else {
      // split the graphs into nth runs of about equal words
      std::vector<std::thread> pool;
      size_t g0 = 0;
      for (size_t t = 0; t < nth && g0 < gs.size(); ++t) {
        const uint64_t until = bwords * (t + 1) / nth;
        size_t g1 = g0;
        while (g1 < gs.size() && (t + 1 == nth || boff[g1] < until)) ++g1;
        if (g1 == g0) g1 = g0 + 1;
        pool.emplace_back(stage, g0, g1);
        g0 = g1;
      }
      for (auto& th : pool) th.join();
      if (g0 < gs.size()) stage(g0, gs.size());
    }
    const uint64_t t0 = steady_ns();  // staging counts as set-up, the copy call as copying
    if (bwords) HIPCHK(hipMemcpyAsync(L.blobs.p, L.pin, bwords * 4, hipMemcpyHostToDevice, st));
    t_copy_ns += steady_ns() - t0;
    t_setup_ns += t0 - t_setup0;
  }
  const uint64_t t_tables0 = steady_ns();
  uint32_t cap32 = 0;
  if ((s = resident_workers(cfg.mapping, cfg.wg_waves, &cap32)) != TG_OK) return s;
  uint32_t nw = cfg.workers ? std::min(cfg.workers, cap32) : cap32;
  const uint32_t G = (uint32_t)gs.size();
  L.gtab_host.assign(G, GraphEnt());
  L.gsrc_host.assign(G, tg::GraphSrc());
  uint64_t N = 0, Pn = 0, E = 0, nsrc = 0, nsinks = 0;
  for (uint32_t gi = 0; gi < G; ++gi) {
    const tg_graph g = gs[gi];
    graph_entry(g, L.gtab_host[gi]);
    tg::GraphSrc& t = L.gsrc_host[gi];
    memset(&t, 0, sizeof(t));
    const uint32_t* b = L.blobs.as<uint32_t>() + boff[gi];
    const tg_graph_s::BlobOff& o = g->bo;
    const bool expl = g->mode == TG_EXPLICIT;
    t.pred_ptr = expl ? b + o.pred_ptr : nullptr;
    t.preds = expl ? b + o.preds : nullptr;
    t.succ_ptr = b + o.succ_ptr;
    t.succ = b + o.succ;
    t.indeg = b + o.indeg;
    t.rounds = b + o.rounds;
    t.slot = o.has_slot ? b + o.slot : nullptr;
    t.req_ptr = expl ? nullptr : b + o.req_ptr;
    t.reqs = expl ? nullptr : (const ReqDev*)(b + o.reqs);
    t.src = b + o.src;
    t.payload = (uint64_t)g->payload.p;
    t.pos_base = (uint32_t)N;
    t.pred_base = (uint32_t)Pn;
    t.succ_base = (uint32_t)E;
    t.src_base = (uint32_t)nsrc;
    t.n = g->n;
    t.mode = g->mode;
    N += g->N();
    Pn += expl ? g->dpred.size() : 0;
    E += g->succ.size();
    nsrc += o.nsrc;
    nsinks += o.nsinks;
  }
  if (N >= 0xFFFFFFF0ull || Pn >= 0xFFFFFFFFull || E >= 0xFFFFFFFFull)
    return fail(TG_EINVAL, "layout too large: %llu tasks, %llu edges", (unsigned long long)N, (unsigned long long)E);
  if (nw > N) nw = N ? (uint32_t)N : 1;
  const uint32_t shards = queue_shards(cfg, nw);
  const uint32_t qwmax = queue_workers_per_shard(cfg, nw, shards);
  const uint64_t cap = N + 64ull * (qwmax + 1);
  // The queue slots the previous launch on this layout filled are emptied
  // (with that launch's geometry) only when the queue buffer is kept: a
  // buffer about to be replaced goes back to the allocator at once, which
  // does not know about work still queued on `st`, so no kernel may be
  // queued against it; its replacement is filled afresh.
  if (L.q.p && L.params.q && L.q.bytes >= (size_t)shards * cap * 4) HIPCHK(tg::launch_queue_clear(L.params, st));
  bool grown = false;
  if ((s = grow(L.rec, N * sizeof(TaskRec))) != TG_OK) return s;
  if ((s = grow(L.pred_addr, Pn * 8)) != TG_OK) return s;
  if ((s = grow(L.succ_pos, E * 4)) != TG_OK) return s;
  if ((s = grow(L.indeg, N * 4)) != TG_OK) return s;
  if ((s = grow(L.cnt, N * 4)) != TG_OK) return s;
  if ((s = grow(L.gtab, G * sizeof(GraphEnt))) != TG_OK) return s;
  if ((s = grow(L.gsrc, G * sizeof(tg::GraphSrc))) != TG_OK) return s;
  if ((s = grow(L.qsrc, nsrc * 4)) != TG_OK) return s;
  if ((s = grow(L.bell, (size_t)nw * tg::kBellStride * 4)) != TG_OK) return s;
  if ((s = grow(L.ctrl, sizeof(tg::Ctrl), &grown)) != TG_OK) return s;
  if (grown) HIPCHK(tg::launch_fill(L.ctrl.as<uint32_t>(), sizeof(tg::Ctrl) / 4, 0, st));
  if ((s = grow(L.q, (size_t)shards * cap * 4, &grown)) != TG_OK) return s;
  if (grown) HIPCHK(tg::launch_fill(L.q.as<uint32_t>(), L.q.bytes / 4, tg::kQEmpty, st));
  const size_t ctl_words = (size_t)(2 * 8 + 1) * tg::kQLine;
  if ((s = grow(L.qctl, ctl_words * 4)) != TG_OK) return s;
  HIPCHK(tg::launch_fill(L.qctl.as<uint32_t>(), ctl_words, 0, st));  // this launch's clear finds nothing to do
  if (G) {
    HIPCHK(hipMemcpyAsync(L.gtab.p, L.gtab_host.data(), G * sizeof(GraphEnt), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(L.gsrc.p, L.gsrc_host.data(), G * sizeof(tg::GraphSrc), hipMemcpyHostToDevice, st));
  }
  if (N || nsrc)
    HIPCHK(tg::launch_build_records(L.gsrc.as<tg::GraphSrc>(), G, (uint32_t)N, (uint32_t)nsrc, L.rec.as<TaskRec>(),
                                    L.pred_addr.as<uint64_t>(), L.succ_pos.as<uint32_t>(), L.indeg.as<uint32_t>(),
                                    L.qsrc.as<uint32_t>(), st));
  L.cfg = cfg;
  L.npos = (uint32_t)N;
  L.nworkers = nw;
  L.grid_blocks = cfg.mapping == TG_MAP_WAVE ? (nw + 3) / 4 : nw;
  L.qwmax = qwmax;
  L.pos_of.clear();
  L.rec_host.clear();
  {
    DevInfo di;
    if ((s = device_info(di)) != TG_OK) return s;
    L.dev = di.dev;
    L.variant = (cfg.mapping == TG_MAP_WAVE ? tg::flight_variant(TG_MAP_WAVE, 1, 1)
                                            : tg::flight_variant(cfg.mapping, cfg.wg_waves, 1)) |
                ((uint64_t)cfg.dispatch << 60);
    L.units = nw;
    L.capacity = cap32;
    if (!L.ev_done) HIPCHK(hipEventCreateWithFlags(&L.ev_done, hipEventDisableTiming));
  }
  ExecParams& P = L.params;
  memset(&P, 0, sizeof(P));
  P.rec = L.rec.as<TaskRec>();
  P.pred_addr = L.pred_addr.as<uint64_t>();
  P.succ_pos = L.succ_pos.as<uint32_t>();
  P.indeg = L.indeg.as<uint32_t>();
  P.cnt = L.cnt.as<uint32_t>();
  P.gtab = L.gtab.as<GraphEnt>();
  P.ctrl = L.ctrl.as<tg::Ctrl>();
  P.bell = L.bell.as<uint32_t>();
  P.gang = 1;
  P.npos = (uint32_t)N;
  P.nworkers = nw;
  P.window = cfg.window;
  P.q = L.q.as<uint32_t>();
  P.qctl = L.qctl.as<uint32_t>();
  P.qsrc = L.qsrc.as<uint32_t>();
  P.nsrc = (uint32_t)nsrc;
  P.nsinks = (uint32_t)nsinks;
  P.qshards = shards;
  P.qcap = (uint32_t)cap;
  P.qtile = cfg.tile;
  P.qsent = cfg.tile * (qwmax + 1);
  if (report && G) {
    // per-graph completion: counts cleared on the stream, flags compared
    // with this launch's sequence number (never cleared)
    if ((s = grow(L.gdone, G * 4)) != TG_OK) return s;
    if (L.gflag_n < G) {
      size_t have = L.gflag_n * 4;
      if ((s = grow_pinned(L.gflag, have, G * 4, true)) != TG_OK) return s;
      L.gflag_n = have / 4;
      memset(L.gflag, 0, L.gflag_n * 4);
      L.gseq = 0;
    }
    HIPCHK(tg::launch_fill(L.gdone.as<uint32_t>(), G, 0, st));
    P.gdone = L.gdone.as<uint32_t>();
    void* dflag = nullptr;
    HIPCHK(hipHostGetDevicePointer(&dflag, L.gflag, 0));
    P.gflag = (uint32_t*)dflag;
    P.gseq = ++L.gseq;
  }
  L.plan_ms = 0;
  L.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_build).count();
  t_tables_ns += steady_ns() - t_tables0;
  return TG_OK;
}

// CPU model of the persistent worker loop: the same state machine as the
// kernels' next_task (ready window of `window` entries, ready tasks taken in
// list order, window slid past the finished prefix), used to check a layout
// for exactly-once execution, precedence and freedom from deadlock without a
// GPU.  Workers take steps in a seeded pseudo-random order; a step either
// runs one task or performs one empty scan.
tg_status emulate_layout(const HostLayout& H, uint32_t window, uint64_t seed, uint32_t* order, uint64_t* executed) {
  const uint32_t N = H.N, nw = H.nw;
  struct St {
    uint32_t h = 0;
    uint64_t done = 0, pend = 0;
  };
  std::vector<uint32_t> cnt(H.indeg);
  std::vector<St> st(nw);
  std::vector<uint32_t> active;
  for (uint32_t w = 0; w < nw; ++w)
    if (H.wbase[w + 1] > H.wbase[w]) active.push_back(w);
  uint64_t ex = 0, rng = seed * 0x9E3779B97F4A7C15ull + 1, idle = 0;
  auto scan = [&](uint32_t w) {
    St& x = st[w];
    const uint32_t wb = H.wbase[w], wcnt = H.wbase[w + 1] - wb;
    uint64_t ready = 0;
    for (uint32_t lane = 0; lane < 64; ++lane) {
      const uint32_t idx = x.h + lane;
      const bool valid = lane < window && idx < wcnt && !((x.done >> lane) & 1ull);
      const uint32_t c = cnt[wb + idx < N ? wb + idx : 0];
      const bool prev_taken = lane == 0 || ((x.done >> (lane - 1)) & 1ull);
      if (valid && (c & tg::kPendingMask) == 0 && (!(c & tg::kAfterPrev) || prev_taken)) ready |= 1ull << lane;
    }
    return ready;
  };
  while (!active.empty()) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    const size_t ai = (size_t)(rng % active.size());
    const uint32_t w = active[ai];
    St& x = st[w];
    const uint32_t wb = H.wbase[w], wcnt = H.wbase[w + 1] - wb;
    if (!x.pend) {
      const uint32_t adv = (~x.done == 0ull) ? 64u : (uint32_t)__builtin_ctzll(~x.done);
      x.h += adv;
      x.done = adv >= 64u ? 0ull : (x.done >> adv);
      if (x.h >= wcnt) {
        active[ai] = active.back();
        active.pop_back();
        continue;
      }
      x.pend = scan(w);
      if (!x.pend) {
        if (++idle > 64ull * active.size() + 1024) {
          bool any = false;
          for (uint32_t w2 : active)
            if (st[w2].pend || scan(w2)) any = true;
          if (!any) {
            *executed = ex;
            return fail(TG_ETIMEOUT, "schedule deadlocks after %llu of %u tasks", (unsigned long long)ex, N);
          }
          idle = 0;
        }
        continue;
      }
    }
    idle = 0;
    const uint32_t b = (uint32_t)__builtin_ctzll(x.pend);
    x.pend &= x.pend - 1;
    x.done |= 1ull << b;
    const uint32_t pos = wb + x.h + b;
    const TaskRec& r = H.rec[pos];
    if (order) order[ex] = pos;
    ++ex;
    for (uint32_t j = 0; j < r.nsucc; ++j) {
      uint32_t& c = cnt[H.succ_pos[r.succ_beg + j]];
      if ((c & tg::kPendingMask) == 0)
        return fail(TG_EINVAL, "counter underflow at position %u", H.succ_pos[r.succ_beg + j]);
      --c;
    }
  }
  *executed = ex;
  return ex == N ? TG_OK : fail(TG_EINVAL, "executed %llu of %u tasks", (unsigned long long)ex, N);
}

// CPU model of the gang executor (k_exec_gang): every one of the G members of
// a gang runs the list dispatch over the gang's list on its own (ready window,
// ballot, oldest entry first), a counter starts at in-degree x G and every
// member decrements each out-edge once when it finishes its share, and the
// in-list edge elision is off.  A member's share is two steps -- take, then
// finish -- so other members and gangs interleave with it, in a seeded
// pseudo-random order.  Checks: a member takes a task only after every member
// of each predecessor has finished it, every member runs each entry of its
// list exactly once, no counter underflows, and no interleaving leaves the
// members stuck.  *executed counts finished shares (N x G when all ran).
// With `elide` the model applies the lists' in-list edge elision, which the
// gang executor leaves off: a member may then take the next entry of its list
// before the other members finished the one before it, and the precedence
// check reports that.
tg_status emulate_gang_layout(const HostLayout& H0, uint32_t G, uint32_t window, uint64_t seed, bool elide,
                              uint64_t* executed) {
  HostLayout E;
  if (elide) {
    E = H0;
    elide_list_edges(E);
  }
  const HostLayout& H = elide ? E : H0;
  const uint32_t N = H.N, nw = H.nw;
  const uint32_t kIdle = 0xFFFFFFFFu;
  struct M {
    uint32_t h = 0, run = 0xFFFFFFFFu;
    uint64_t done = 0, pend = 0;
  };
  std::vector<uint32_t> cnt(N), finished(N, 0);
  for (uint32_t p = 0; p < N; ++p) {
    const uint32_t d = H.indeg[p] & tg::kPendingMask;
    if (d > tg::kPendingMask / G) return fail(TG_EINVAL, "in-degree too large for the gang");
    cnt[p] = d * G | (H.indeg[p] & tg::kAfterPrev);
  }
  // predecessors by position (every edge of the graph, elided or not), to
  // check precedence at each take
  std::vector<uint32_t> pptr(N + 1, 0), pred;
  for (uint32_t p = 0; p < N; ++p)
    for (uint32_t j = 0; j < H0.rec[p].nsucc; ++j) pptr[H0.succ_pos[H0.rec[p].succ_beg + j] + 1]++;
  for (uint32_t p = 0; p < N; ++p) pptr[p + 1] += pptr[p];
  pred.resize(pptr[N]);
  {
    std::vector<uint32_t> fill(pptr.begin(), pptr.end() - 1);
    for (uint32_t p = 0; p < N; ++p)
      for (uint32_t j = 0; j < H0.rec[p].nsucc; ++j) pred[fill[H0.succ_pos[H0.rec[p].succ_beg + j]]++] = p;
  }
  std::vector<M> mem((size_t)nw * G);
  std::vector<uint32_t> active;
  for (uint32_t w = 0; w < nw; ++w)
    if (H.wbase[w + 1] > H.wbase[w])
      for (uint32_t m = 0; m < G; ++m) active.push_back(w * G + m);
  uint64_t ex = 0, rng = seed * 0x9E3779B97F4A7C15ull + 1, idle = 0;
  auto scan = [&](uint32_t a) {
    const M& x = mem[a];
    const uint32_t w = a / G, wb = H.wbase[w], wcnt = H.wbase[w + 1] - wb;
    uint64_t ready = 0;
    for (uint32_t lane = 0; lane < 64; ++lane) {
      const uint32_t idx = x.h + lane;
      const bool valid = lane < window && idx < wcnt && !((x.done >> lane) & 1ull);
      const uint32_t c = cnt[wb + idx < N ? wb + idx : 0];
      const bool prev_taken = lane == 0 || ((x.done >> (lane - 1)) & 1ull);
      if (valid && (c & tg::kPendingMask) == 0 && (!(c & tg::kAfterPrev) || prev_taken)) ready |= 1ull << lane;
    }
    return ready;
  };
  while (!active.empty()) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    const size_t ai = (size_t)(rng % active.size());
    const uint32_t a = active[ai];
    M& x = mem[a];
    const uint32_t w = a / G, wb = H.wbase[w], wcnt = H.wbase[w + 1] - wb;
    if (x.run != kIdle) {  // finish this member's share
      const TaskRec& r = H.rec[x.run];
      for (uint32_t j = 0; j < r.nsucc; ++j) {
        uint32_t& c = cnt[H.succ_pos[r.succ_beg + j]];
        if ((c & tg::kPendingMask) == 0)
          return fail(TG_EINVAL, "counter underflow at position %u", H.succ_pos[r.succ_beg + j]);
        --c;
      }
      if (++finished[x.run] > G) return fail(TG_EINVAL, "position %u finished more than %u times", x.run, G);
      x.run = kIdle;
      ++ex;
      idle = 0;
      continue;
    }
    if (!x.pend) {
      const uint32_t adv = (~x.done == 0ull) ? 64u : (uint32_t)__builtin_ctzll(~x.done);
      x.h += adv;
      x.done = adv >= 64u ? 0ull : (x.done >> adv);
      if (x.h >= wcnt) {
        active[ai] = active.back();
        active.pop_back();
        continue;
      }
      x.pend = scan(a);
      if (!x.pend) {
        if (++idle > 64ull * active.size() + 1024) {
          bool any = false;
          for (uint32_t a2 : active)
            if (mem[a2].pend || mem[a2].run != kIdle || scan(a2)) any = true;
          if (!any) {
            *executed = ex;
            return fail(TG_ETIMEOUT, "gang schedule deadlocks after %llu of %llu shares", (unsigned long long)ex,
                        (unsigned long long)N * G);
          }
          idle = 0;
        }
        continue;
      }
    }
    idle = 0;
    const uint32_t b = (uint32_t)__builtin_ctzll(x.pend);
    x.pend &= x.pend - 1;
    x.done |= 1ull << b;
    const uint32_t pos = wb + x.h + b;
    for (uint32_t i = pptr[pos]; i < pptr[pos + 1]; ++i)
      if (finished[pred[i]] != G)
        return fail(TG_EINVAL, "position %u taken before its predecessor %u finished", pos, pred[i]);
    x.run = pos;
  }
  *executed = ex;
  for (uint32_t p = 0; p < N; ++p)
    if (finished[p] != G) return fail(TG_EINVAL, "position %u finished %u of %u times", p, finished[p], G);
  return TG_OK;
}

// CPU model of the ready-queue dispatch (k_exec_wave_q): workers take one
// step at a time in a seeded pseudo-random order, and every access to shared
// state is a step of its own, so the model visits the interleavings the
// kernels can produce -- a claim's atomic add on a shard head, polls of a
// claimed slot that is still empty, a push's reservation of tickets on a
// shard tail and each write of a reserved slot, the report of finished sinks,
// and the finisher's reservation and writes of the exit sentinels.  It checks
// that every task runs exactly once, after all its in-edges, that no ticket
// lies beyond a shard's capacity (the task count plus the sentinels), that a
// worker leaves only after reporting its sinks, and that every worker leaves.
tg_status emulate_queue(const HostLayout& H, uint32_t nworkers, uint32_t shards, uint32_t tile, uint64_t seed,
                        uint32_t* order, uint64_t* executed) {
  const uint32_t N = H.N;
  const uint32_t kNone = 0xFFFFFFFFu, kExitSlot = 0xFFFFFFFEu;
  Config qc;
  qc.mapping = TG_MAP_WAVE;
  qc.shards = shards;
  shards = queue_shards(qc, nworkers);
  const uint32_t wmax = queue_workers_per_shard(qc, nworkers, shards);
  const uint64_t cap = (uint64_t)N + 64ull * (wmax + 1);
  const uint32_t sent = tile * (wmax + 1);
  std::vector<uint32_t> cnt(H.indeg);
  std::vector<std::vector<uint32_t>> slot(shards, std::vector<uint32_t>(cap, kNone));
  std::vector<uint64_t> head(shards, 0), tail(shards, 0);
  uint32_t nsrc = 0, nsinks = 0;
  for (uint32_t p = 0; p < N; ++p) {
    if (H.indeg[p] == 0) {
      slot[nsrc % shards][nsrc / shards] = p;
      nsrc++;
    }
    if (H.rec[p].nsucc == 0) ++nsinks;
  }
  for (uint32_t s = 0; s < shards; ++s) tail[s] = (nsrc + shards - 1 - s) / shards;
  uint64_t fin = 0, ex = 0;
  std::vector<uint8_t> done(N, 0);
  enum Phase { kNext, kClaim, kPoll, kReport, kReserve, kWrite, kFinReserve, kFinWrite };
  struct W {
    Phase ph = kNext;
    uint32_t shard = 0, pshard = 0, local = 0xFFFFFFFFu;
    uint64_t tile_h = 0;
    uint32_t tile_n = 0, tile_i = 0, sinks = 0;
    std::vector<uint32_t> pending;  // ready positions to write into reserved slots
    uint64_t pbase = 0;
    uint32_t ps = 0, fin_s = 0, fin_left = 0;
  };
  std::vector<W> ws(nworkers);
  for (uint32_t w = 0; w < nworkers; ++w) ws[w].shard = ws[w].pshard = ((w / 4) & 7u) & (shards - 1u);
  uint64_t rng = seed * 0x9E3779B97F4A7C15ull + 7;
  auto next_rand = [&]() {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
  };
  // run task `pos` on worker x: signal its out-edges, keep one ready successor
  auto run = [&](W& x, uint32_t pos) -> tg_status {
    if (pos >= N || done[pos] || cnt[pos] != 0) return fail(TG_EINVAL, "queue model: position %u run twice or early", pos);
    done[pos] = 1;
    if (order) order[ex] = pos;
    ++ex;
    const TaskRec& r = H.rec[pos];
    if (r.nsucc == 0) x.sinks++;
    std::vector<uint32_t> ready;
    for (uint32_t j = 0; j < r.nsucc; ++j) {
      const uint32_t d = H.succ_pos[r.succ_beg + j];
      if (cnt[d] == 0) return fail(TG_EINVAL, "queue model: counter underflow at %u", d);
      if (--cnt[d] == 0) ready.push_back(d);
    }
    if (!ready.empty() && x.local == kNone) {
      x.local = ready.front();
      ready.erase(ready.begin());
    }
    x.pending.assign(ready.rbegin(), ready.rend());
    x.ph = x.pending.empty() ? kNext : kReserve;
    return TG_OK;
  };
  std::vector<uint32_t> live(nworkers);
  for (uint32_t w = 0; w < nworkers; ++w) live[w] = w;
  uint64_t steps = 0;
  const uint64_t max_steps = 64ull * (N + 16) * (nworkers + 8) + 100000;
  tg_status st = TG_OK;
  while (!live.empty()) {
    if (++steps > max_steps) {
      *executed = ex;
      return fail(TG_ETIMEOUT, "queue model does not terminate after %llu of %u tasks", (unsigned long long)ex, N);
    }
    const size_t li = (size_t)(next_rand() % live.size());
    W& x = ws[live[li]];
    switch (x.ph) {
      case kNext:
        if (x.local != kNone) {
          const uint32_t pos = x.local;
          x.local = kNone;
          if ((st = run(x, pos)) != TG_OK) return st;
        } else {
          x.ph = x.tile_i == x.tile_n ? kClaim : kPoll;
        }
        break;
      case kClaim:  // one atomic add on the head: never fails
        x.tile_h = head[x.shard];
        head[x.shard] += tile;
        x.tile_n = tile;
        x.tile_i = 0;
        x.ph = kPoll;
        break;
      case kPoll: {
        const uint64_t t = x.tile_h + x.tile_i;
        if (t >= cap) return fail(TG_EINVAL, "queue model: ticket %llu beyond capacity %llu", (unsigned long long)t,
                                  (unsigned long long)cap);
        const uint32_t v = slot[x.shard][t];
        if (v == kNone) {
          if (x.sinks) x.ph = kReport;  // nothing to run: report finished sinks first
          break;
        }
        x.tile_i++;
        if (v == kExitSlot) {
          if (x.sinks) return fail(TG_EINVAL, "queue model: worker leaves with unreported sinks");
          live[li] = live.back();
          live.pop_back();
          break;
        }
        if ((st = run(x, v)) != TG_OK) return st;
        break;
      }
      case kReport: {
        const uint64_t old = fin;
        fin += x.sinks;
        const bool last = old + x.sinks == nsinks;
        x.sinks = 0;
        if (last) {
          x.fin_s = 0;
          x.ph = kFinReserve;
        } else {
          x.ph = kPoll;
        }
        break;
      }
      case kFinReserve:
        x.pbase = tail[x.fin_s];
        tail[x.fin_s] += sent;
        x.fin_left = sent;
        x.ph = kFinWrite;
        break;
      case kFinWrite:
        if (x.pbase >= cap) return fail(TG_EINVAL, "queue model: sentinel beyond capacity");
        slot[x.fin_s][x.pbase++] = kExitSlot;
        if (--x.fin_left == 0) x.ph = ++x.fin_s < shards ? kFinReserve : kPoll;
        break;
      case kReserve:
        x.ps = x.pshard;
        x.pshard = (x.pshard + 1) % shards;
        x.pbase = tail[x.ps];
        tail[x.ps] += x.pending.size();
        if (tail[x.ps] > cap) return fail(TG_EINVAL, "queue model: shard %u overflows", x.ps);
        x.ph = kWrite;
        break;
      case kWrite:
        slot[x.ps][x.pbase++] = x.pending.back();
        x.pending.pop_back();
        if (x.pending.empty()) x.ph = kNext;
        break;
    }
  }
  *executed = ex;
  if (ex != N) return fail(TG_EINVAL, "queue model ran %llu of %u tasks", (unsigned long long)ex, N);
  if (fin != nsinks) return fail(TG_EINVAL, "queue model: %llu of %u sinks reported", (unsigned long long)fin, nsinks);
  return TG_OK;
}

// Timed model of a layout: every worker runs the kernels' ready-window rule
// (first ready entry of its window, window slid past the finished prefix)
// with each task taking its estimated cost; an idle worker wakes when one of
// its tasks becomes ready.  Returns the simulated makespan in cost units and
// the lower bound max(longest path, total cost / workers).
void timed_makespan(const std::vector<tg_graph>& gs, const HostLayout& H, uint32_t window, uint64_t* makespan,
                    uint64_t* bound) {
  const uint32_t N = H.N, nw = H.nw;
  std::vector<uint64_t> cost(N);
  std::vector<uint32_t> owner(N);
  uint64_t total = 0;
  for (uint32_t gi = 0; gi < gs.size(); ++gi)
    for (uint32_t v = 0; v < gs[gi]->N(); ++v) {
      const uint32_t pos = H.pos_of[gi][v];
      cost[pos] = task_cost(gs[gi], v);
      total += cost[pos];
    }
  for (uint32_t w = 0; w < nw; ++w)
    for (uint32_t p = H.wbase[w]; p < H.wbase[w + 1]; ++p) owner[p] = w;
  // longest path (positions' records hold the successors)
  std::vector<uint64_t> est(N, 0);
  uint64_t cp = 0;
  {
    std::vector<uint32_t> cnt(H.indeg), q;
    for (uint32_t p = 0; p < N; ++p)
      if (!cnt[p]) q.push_back(p);
    for (size_t i = 0; i < q.size(); ++i) {
      const uint32_t p = q[i];
      const uint64_t f = est[p] + cost[p];
      cp = std::max(cp, f);
      const TaskRec& r = H.rec[p];
      for (uint32_t j = 0; j < r.nsucc; ++j) {
        const uint32_t d = H.succ_pos[r.succ_beg + j];
        est[d] = std::max(est[d], f);
        if (--cnt[d] == 0) q.push_back(d);
      }
    }
  }
  *bound = std::max(cp, (total + nw - 1) / nw);
  struct W {
    uint32_t h = 0;
    uint64_t done = 0;
    bool idle = false;
  };
  std::vector<W> ws(nw);
  std::vector<uint32_t> cnt(H.indeg);
  typedef std::pair<uint64_t, uint64_t> Ev;  // (time, kind << 32 | id): kind 0 = finish(pos), 1 = wake(worker)
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> evq;
  for (uint32_t w = 0; w < nw; ++w) evq.push(Ev(0, (1ull << 32) | w));
  uint64_t t_end = 0;
  while (!evq.empty()) {
    const Ev e = evq.top();
    evq.pop();
    const uint64_t t = e.first;
    const uint32_t id = (uint32_t)e.second;
    if ((e.second >> 32) == 0) {
      t_end = std::max(t_end, t);
      const TaskRec& r = H.rec[id];
      for (uint32_t j = 0; j < r.nsucc; ++j) {
        const uint32_t d = H.succ_pos[r.succ_beg + j];
        if (--cnt[d] == 0 && ws[owner[d]].idle) {
          ws[owner[d]].idle = false;
          evq.push(Ev(t, (1ull << 32) | owner[d]));
        }
      }
      evq.push(Ev(t, (1ull << 32) | owner[id]));  // the worker is free again
      continue;
    }
    W& x = ws[id];
    const uint32_t wb = H.wbase[id], wcnt = H.wbase[id + 1] - wb;
    const uint32_t adv = (~x.done == 0ull) ? 64u : (uint32_t)__builtin_ctzll(~x.done);
    x.h += adv;
    x.done = adv >= 64u ? 0ull : (x.done >> adv);
    if (x.h >= wcnt) continue;
    bool ran = false;
    for (uint32_t lane = 0; lane < window && x.h + lane < wcnt; ++lane) {
      if ((x.done >> lane) & 1ull) continue;
      const uint32_t p = wb + x.h + lane;
      if (cnt[p] != 0) continue;
      x.done |= 1ull << lane;
      cnt[p] = 0xFFFFFFFFu;  // taken
      evq.push(Ev(t + cost[p], (uint64_t)p));
      ran = true;
      break;
    }
    if (!ran) x.idle = true;
  }
  *makespan = t_end;
}

bool same_layout(const Config& a, const Config& b) {
  return a.mapping == b.mapping && a.workers == b.workers && a.wg_waves == b.wg_waves && a.schedule == b.schedule &&
         a.gang == b.gang && a.dispatch == b.dispatch && (a.dispatch == TG_DISPATCH_LISTS || a.shards == b.shards);
}

// Launch reset + persistent executor for a layout.  Under the ledger lock:
// drop finished launches, make `st` wait for the in-flight launches this one
// cannot overlap (tg_ledger.h), issue the kernels, record the completion
// event and enter the launch.
// External conditions of one launch: pre-condition flags checked on the
// device before the executor starts, and a flag set on the device after it.
struct LaunchConds {
  tg::FlagWait pre{};
  uint32_t* post = nullptr;  // device address of the post-condition flag, or null
  uint32_t post_value = 0;
};

tg_status launch_layout(Layout& L, const Config& cfg, const std::vector<tg_graph>& gs, hipStream_t st,
                        hipEvent_t before_kernel = nullptr, hipEvent_t ring0 = nullptr, hipEvent_t ring1 = nullptr,
                        const LaunchConds* conds = nullptr) {
  std::lock_guard<std::mutex> ledger_lk(g_ledger_mu);
  for (size_t i = 0; i < g_flights.size();) {
    if (g_flights[i].key != &L && hipEventQuery(g_flight_ev[i]) == hipErrorNotReady) {
      ++i;
      continue;
    }
    g_flights.erase(g_flights.begin() + (ptrdiff_t)i);
    g_flight_ev.erase(g_flight_ev.begin() + (ptrdiff_t)i);
  }
  (void)hipGetLastError();  // a not-ready query is not an error of this launch
  tg::Flight me;
  me.key = &L;
  me.dev = L.dev;
  me.variant = L.variant;
  me.workers = L.units;
  me.capacity = L.capacity;
  me.stream = (uintptr_t)st;
  for (size_t i : tg::flights_to_follow(g_flights, me)) HIPCHK(hipStreamWaitEvent(st, g_flight_ev[i], 0));
  ExecParams P = L.params;
  P.window = cfg.window;
  P.spin_limit = cfg.spin_limit;
  P.diag = cfg.diag;
  P.idle_sleep = cfg.idle_sleep;
  P.notify = cfg.notify;
  P.watchdog_ticks = (uint64_t)cfg.watchdog_ms * 100000ull;
  P.progress_ticks = P.watchdog_ticks / 16;
  P.execs = nullptr;
  P.wprog = nullptr;
  P.tstamp = nullptr;
  P.wstamp = nullptr;
  if (cfg.diag) {
    tg_status s;
    if (!L.execs.p && (s = L.execs.alloc((size_t)L.npos * 4)) != TG_OK) return s;
    if (!L.wprog.p && (s = L.wprog.alloc((size_t)L.nworkers * 4)) != TG_OK) return s;
    if (!L.tstamp.p && (s = L.tstamp.alloc((size_t)L.npos * 16)) != TG_OK) return s;
    if (!L.wstamp.p && (s = L.wstamp.alloc((size_t)L.nworkers * 32)) != TG_OK) return s;
    P.execs = L.execs.as<uint32_t>();
    P.wprog = L.wprog.as<uint32_t>();
    P.tstamp = L.tstamp.as<uint64_t>();
    P.wstamp = L.wstamp.as<uint64_t>();
  }
  for (auto g : gs)
    if (g->mode == TG_IMPLICIT) {
      HIPCHK(tg_launch_init_data(g->data.as<uint32_t>(), g->space, sm64_host(g->seed ^ (2ull << 32)), st));
    }
  const bool queue = L.cfg.dispatch == TG_DISPATCH_QUEUE;
  if (queue) {
    P.qtile = cfg.tile;
    P.qsent = cfg.tile * (L.qwmax + 1);
  }
  HIPCHK(tg::launch_reset(P, st));
  if (queue) HIPCHK(tg::launch_queue_reset(P, st));
  P.gated = conds && conds->pre.n ? 1u : 0u;
  if (P.gated) HIPCHK(tg::launch_wait_flags(conds->pre, P.ctrl, P.watchdog_ticks, st));
  if (before_kernel) HIPCHK(hipEventRecord(before_kernel, st));
  if (ring0) HIPCHK(hipEventRecord(ring0, st));
  if (L.npos) {
    if (queue) HIPCHK(tg::launch_exec_queue(P, cfg.mapping, cfg.wg_waves, L.grid_blocks, st));
    else HIPCHK(tg::launch_exec(P, cfg.mapping, cfg.wg_waves, L.grid_blocks, st));
  }
  if (ring1) HIPCHK(hipEventRecord(ring1, st));
  if (conds && conds->post) HIPCHK(tg::launch_set_flag(conds->post, conds->post_value, P.ctrl, st));
  HIPCHK(hipEventRecord(L.ev_done, st));
  g_flights.push_back(me);
  g_flight_ev.push_back(L.ev_done);
  return TG_OK;
}

tg_status check_abort(Layout* L) {
  if (!L) return TG_OK;
  tg::Ctrl c;
  HIPCHK(hipMemcpy(&c, L->ctrl.p, sizeof(c), hipMemcpyDeviceToHost));
  L->last_started = c.started;
  if (c.sticky || c.abort) {
    // the host has now seen these aborts: clear them so the next counter
    // reset does not carry them forward
    const uint32_t zero[2] = {0, 0};
    HIPCHK(hipMemcpy(&L->ctrl.as<tg::Ctrl>()->sticky, zero, 8, hipMemcpyHostToDevice));  // sticky, precond
    HIPCHK(hipMemcpy(&L->ctrl.as<tg::Ctrl>()->abort, zero, 4, hipMemcpyHostToDevice));
    tg_status s = null_stream_fence();
    if (s != TG_OK) return s;
  }
  if (c.abort && c.precond)
    return fail(TG_ETIMEOUT, "pre-condition flag %u was not met within the watchdog interval: no task ran",
                c.precond - 1);
  if (c.abort)
    return fail(TG_ETIMEOUT,
                "executor watchdog aborted the launch (no progress): worker %u of %u stuck at list entry %u/%u "
                "(position %u, pending in-edges %u)",
                c.stuck_worker, L->nworkers, c.stuck_h, c.stuck_wcnt, c.stuck_pos, c.stuck_cnt & tg::kPendingMask);
  if (c.sticky) return fail(TG_ETIMEOUT, "an earlier launch of this layout was aborted by the executor watchdog");
  return TG_OK;
}

tg_status graph_wait(tg_graph g) {
  if (!g->inflight) return TG_OK;
  g->inflight = false;
  HIPCHK(hipEventSynchronize(g->ev1));
  float ms = 0;
  if (hipEventElapsedTime(&ms, g->ev0, g->ev1) == hipSuccess) g->exec_ms = ms;
  g->kernel_ms = 0;
  if (g->last_layout && hipEventElapsedTime(&ms, g->evk, g->ev1) == hipSuccess) g->kernel_ms = ms;
  (void)hipGetLastError();
  return check_abort(g->last_layout);
}

// Buffer lifetimes (payload slots).  Algorithm 1 starts a vertex when the
// counter of its pending in-edges reaches zero; the same counters can order
// the reuse of payload memory.  Tasks are visited in dependence-level order
// (ties by id).  When the last consumer of a task p has been visited, p's
// slot becomes free for tasks of a later level than that consumer; under
// TG_KEEP_NONE a task without consumers frees its slot at once.  A task
// takes the oldest free slot it may use (else a new one), and for each task
// whose reads of the slot's previous contents must finish first (the
// previous owner's consumers, or the previous owner itself if it had none)
// an anti-dependence edge to the new owner is added to the executed edges.
// Every such edge goes from a lower to a higher level, so the levels, the
// critical path and the schedules' level order are unchanged, and a payload
// is overwritten only after every task that reads it has finished.
void assign_slots(tg_graph g) {
  const uint32_t N = g->N();
  uint32_t maxlevel = 0;
  for (uint32_t lv : g->level) maxlevel = std::max(maxlevel, lv);
  std::vector<uint64_t> lstart((size_t)maxlevel + 2, 0);
  for (uint32_t lv : g->level) lstart[lv + 1]++;
  for (size_t i = 1; i < lstart.size(); ++i) lstart[i] += lstart[i - 1];
  g->topo.assign(N, 0);
  for (uint32_t v = 0; v < N; ++v) g->topo[lstart[g->level[v]]++] = v;
  struct Freed {
    uint32_t slot, min_level, by;
    bool self;  // by itself (a task without consumers), else by's consumers
  };
  std::deque<Freed> freeq;
  std::vector<uint32_t> remaining(N);
  for (uint32_t v = 0; v < N; ++v) remaining[v] = (uint32_t)(g->succ_ptr[v + 1] - g->succ_ptr[v]);
  g->slot_of.assign(N, 0);
  g->slot_last.clear();
  std::vector<std::pair<uint32_t, uint32_t>> extra;  // anti-dependence edges (from, to)
  for (uint32_t v : g->topo) {
    uint32_t slot;
    if (!freeq.empty() && freeq.front().min_level <= g->level[v]) {
      const Freed f = freeq.front();
      freeq.pop_front();
      slot = f.slot;
      if (f.self) {
        extra.emplace_back(f.by, v);
      } else {
        for (uint64_t j = g->succ_ptr[f.by]; j < g->succ_ptr[f.by + 1]; ++j) extra.emplace_back(g->succ[j], v);
      }
    } else {
      slot = (uint32_t)g->slot_last.size();
      g->slot_last.push_back(v);
    }
    g->slot_of[v] = slot;
    g->slot_last[slot] = v;
    for (uint64_t j = g->dpred_ptr[v]; j < g->dpred_ptr[v + 1]; ++j) {
      const uint32_t p = g->dpred[j];
      if (--remaining[p] == 0) freeq.push_back(Freed{g->slot_of[p], g->level[v] + 1, p, false});
    }
    if (g->retain == TG_KEEP_NONE && g->succ_ptr[v + 1] == g->succ_ptr[v])
      freeq.push_back(Freed{slot, g->level[v] + 1, v, true});
  }
  g->nslots = (uint32_t)g->slot_last.size();
  // executed edges: data edges plus the anti-dependence edges not already
  // among them, rows ascending
  std::vector<std::pair<uint32_t, uint32_t>> all;
  all.reserve(g->succ.size() + extra.size());
  for (uint32_t u = 0; u < N; ++u)
    for (uint64_t j = g->succ_ptr[u]; j < g->succ_ptr[u + 1]; ++j) all.emplace_back(u, g->succ[j]);
  all.insert(all.end(), extra.begin(), extra.end());
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  g->full_succ_ptr = g->succ_ptr;
  g->full_succ = g->succ;
  g->succ_ptr.assign((size_t)N + 1, 0);
  g->succ.resize(all.size());
  std::fill(g->xindeg.begin(), g->xindeg.end(), 0u);
  for (size_t i = 0; i < all.size(); ++i) {
    g->succ_ptr[all[i].first + 1]++;
    g->succ[i] = all[i].second;
    g->xindeg[all[i].second]++;
  }
  for (uint32_t u = 0; u < N; ++u) g->succ_ptr[u + 1] += g->succ_ptr[u];
  g->anti = true;  // the executed edges are kept apart from the data edges
}

tg_status finalize_explicit(tg_graph g) {
  const uint32_t N = g->N();
  // distinct predecessor sets
  g->dpred_ptr.assign((size_t)N + 1, 0);
  g->dpred.clear();
  g->dpred.reserve(g->preds.size());
  std::vector<uint32_t> tmp;
  for (uint32_t v = 0; v < N; ++v) {
    tmp.assign(g->preds.begin() + g->pred_ptr[v], g->preds.begin() + g->pred_ptr[v + 1]);
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    g->dpred.insert(g->dpred.end(), tmp.begin(), tmp.end());
    g->dpred_ptr[v + 1] = g->dpred.size();
  }
  // out-edge CSR, rows ascending (ids are appended in increasing v)
  g->succ_ptr.assign((size_t)N + 1, 0);
  for (uint32_t p : g->dpred) g->succ_ptr[p + 1]++;
  for (uint32_t v = 0; v < N; ++v) g->succ_ptr[v + 1] += g->succ_ptr[v];
  g->succ.assign(g->dpred.size(), 0);
  {
    std::vector<uint64_t> fill(g->succ_ptr.begin(), g->succ_ptr.end() - 1);
    for (uint32_t v = 0; v < N; ++v)
      for (uint64_t j = g->dpred_ptr[v]; j < g->dpred_ptr[v + 1]; ++j) g->succ[fill[g->dpred[j]]++] = v;
  }
  // dependence levels (creation order is topological)
  g->level.assign(N, 0);
  for (uint32_t v = 0; v < N; ++v) {
    uint32_t lv = 0;
    for (uint64_t j = g->dpred_ptr[v]; j < g->dpred_ptr[v + 1]; ++j) lv = std::max(lv, g->level[g->dpred[j]] + 1);
    g->level[v] = lv;
  }
  g->xindeg.resize(N);
  for (uint32_t v = 0; v < N; ++v) g->xindeg[v] = (uint32_t)(g->dpred_ptr[v + 1] - g->dpred_ptr[v]);
  g->nslots = N;
  if (g->retain != TG_KEEP_ALL) assign_slots(g);
  return TG_OK;
}

// Packs the compiled graph into g->blob (see tg_graph_s::BlobOff): rows of
// distinct predecessors (explicit) and of executed successors as u32
// offsets, counter reset values, mix rounds, payload slots, requirement rows
// and requirements (implicit, 32-byte ReqDev records), and the sources.
// Called whenever any of these change after finalize.
tg_status build_blob(tg_graph g) {
  const uint32_t N = g->N();
  const bool expl = g->mode == TG_EXPLICIT;
  const uint64_t P = expl ? g->dpred.size() : 0, E = g->succ.size(), M = expl ? 0 : g->reqs.size();
  if (P >= 0xFFFFFFFFull || E >= 0xFFFFFFFFull || M >= 0xFFFFFFFFull)
    return fail(TG_EINVAL, "graph too large for 32-bit edge offsets");
  tg_graph_s::BlobOff o;
  uint64_t w = 0;
  auto take = [&](uint64_t words) {  // sections start on 32-byte boundaries
    const uint64_t at = w;
    w += (words + 7) & ~7ull;
    return at;
  };
  for (uint32_t v = 0; v < N; ++v) {
    if (g->xindeg[v] == 0) o.nsrc++;
    if (g->succ_ptr[v + 1] == g->succ_ptr[v]) o.nsinks++;
  }
  o.has_slot = expl && !g->slot_of.empty();
  if (expl) {
    o.pred_ptr = take((uint64_t)N + 1);
    o.preds = take(P);
  } else {
    o.req_ptr = take((uint64_t)N + 1);
    o.reqs = take(M * (sizeof(ReqDev) / 4));
  }
  o.succ_ptr = take((uint64_t)N + 1);
  o.succ = take(E);
  o.indeg = take(N);
  o.rounds = take(N);
  if (o.has_slot) o.slot = take(N);
  o.src = take(o.nsrc);
  o.words = w;
  std::vector<uint32_t>& b = g->blob;
  b.assign(w, 0);
  if (expl) {
    for (uint32_t v = 0; v <= N; ++v) b[o.pred_ptr + v] = (uint32_t)g->dpred_ptr[v];
    std::copy(g->dpred.begin(), g->dpred.end(), b.begin() + o.preds);
  } else {
    for (uint32_t v = 0; v <= N; ++v) b[o.req_ptr + v] = (uint32_t)g->req_ptr[v];
    for (uint64_t i = 0; i < M; ++i) {
      ReqDev q;
      memset(&q, 0, sizeof(q));
      q.lo = g->reqs[i].lo;
      q.hi = g->reqs[i].hi;
      q.priv = g->reqs[i].priv;
      q.rw_base = g->rw_base[i];
      memcpy(b.data() + o.reqs + i * (sizeof(ReqDev) / 4), &q, sizeof(q));
    }
  }
  for (uint32_t v = 0; v <= N; ++v) b[o.succ_ptr + v] = (uint32_t)g->succ_ptr[v];
  std::copy(g->succ.begin(), g->succ.end(), b.begin() + o.succ);
  std::copy(g->xindeg.begin(), g->xindeg.end(), b.begin() + o.indeg);
  std::copy(g->rounds.begin(), g->rounds.end(), b.begin() + o.rounds);
  if (o.has_slot) std::copy(g->slot_of.begin(), g->slot_of.end(), b.begin() + o.slot);
  for (uint32_t v = 0, k = 0; v < N; ++v)
    if (g->xindeg[v] == 0) b[o.src + k++] = v;
  g->bo = o;
  g->blob_gen++;
  return TG_OK;
}

// Uploads the compiled graph's blob if the device copy is missing or stale
// (on `st`; the null stream when st is null).
tg_status ensure_blob(tg_graph g, hipStream_t st) {
  if (g->dblob.p && g->dblob_gen == g->blob_gen) return TG_OK;
  tg_status s;
  const size_t bytes = std::max<size_t>(g->blob.size(), 8) * 4;
  if (g->dblob.p && g->dblob.bytes < bytes) g->dblob.release();
  if (!g->dblob.p) {
    if ((s = g->dblob.alloc(bytes)) != TG_OK) return s;
    g->dev_gen++;  // layouts hold addresses inside it
  }
  const uint64_t t0 = steady_ns();
  if (!g->blob.empty()) HIPCHK(hipMemcpyAsync(g->dblob.p, g->blob.data(), g->blob.size() * 4, hipMemcpyHostToDevice, st));
  t_copy_ns += steady_ns() - t0;
  g->dblob_gen = g->blob_gen;
  return TG_OK;
}

// Device address of task v's first requirement (implicit graphs).
uint64_t req_addr(tg_graph g, uint32_t v) {
  return (uint64_t)g->dblob.p + (g->bo.reqs + (uint64_t)g->blob[g->bo.req_ptr + v] * (sizeof(ReqDev) / 4)) * 4;
}

// Device buffers of a graph are allocated on first use, so graphs can be
// built and compiled on a machine without a GPU.
tg_status ensure_device(tg_graph g, bool upload_blob) {
  const uint32_t N = g->N();
  tg_status s;
  g->released = false;
  if ((g->mode == TG_EXPLICIT && !g->payload.p) || (g->mode == TG_IMPLICIT && !g->data.p) || !g->digest.p) g->dev_gen++;
  if (g->mode == TG_EXPLICIT && !g->payload.p) {
    if ((s = g->payload.alloc((size_t)g->nslots * g->n * 4)) != TG_OK) return s;
  }
  if (g->mode == TG_IMPLICIT && !g->data.p) {
    if ((s = g->data.alloc((size_t)g->space * 4)) != TG_OK) return s;
  }
  if (!g->digest.p) {
    if ((s = g->digest.alloc((size_t)N * 4)) != TG_OK) return s;
    HIPCHK(hipMemsetAsync(g->digest.p, 0, (size_t)N * 4, t_copy_stream));
  }
  if (upload_blob && (s = ensure_blob(g, t_copy_stream)) != TG_OK) return s;
  return TG_OK;  // the caller fences the null stream once for all its graphs
}

// Timing events of a graph's own launches, created at its first one (graphs
// that only ever run inside batches or the server never need them).
// The comparator's hipGraph copies the solo layout's device addresses (task
// records, graph table, positions) into its kernel nodes, so it must never
// outlive that layout: every place that replaces or releases the solo
// layout goes through here, after the graph's executions have finished.
void drop_solo(tg_graph g) {
  if (g->hgx) (void)hipGraphExecDestroy(g->hgx);
  if (g->hg) (void)hipGraphDestroy(g->hg);
  if (g->hgcx) (void)hipGraphExecDestroy(g->hgcx);
  if (g->hgc) (void)hipGraphDestroy(g->hgc);
  g->hgx = g->hgcx = nullptr;
  g->hg = g->hgc = nullptr;
  g->solo.reset();
  g->last_layout = nullptr;
}

tg_status ensure_events(tg_graph g) {
  if (!g->ev0) HIPCHK(hipEventCreate(&g->ev0));
  if (!g->ev1) HIPCHK(hipEventCreate(&g->ev1));
  if (!g->evk) HIPCHK(hipEventCreate(&g->evk));
  if (!g->rk0[0])
    for (uint32_t i = 0; i < tg_graph_s::kRing; ++i) {
      HIPCHK(hipEventCreate(&g->rk0[i]));
      HIPCHK(hipEventCreate(&g->rk1[i]));
    }
  return TG_OK;
}

}  // namespace

// Implicit mode: infer the conflict DAG on the device, then derive the
// predecessor sets and levels on the host exactly as for explicit graphs.
static tg_status tg_finalize_implicit(tg_graph g) {
  const uint32_t N = g->N();
  // ordinal of each read-write interval's first element among its task's
  // written elements (digest weights follow declaration order)
  g->rw_base.assign(g->reqs.size(), 0);
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t run = 0;
    for (uint64_t a = g->req_ptr[k]; a < g->req_ptr[k + 1]; ++a) {
      g->rw_base[a] = (uint32_t)run;
      if (g->reqs[a].priv == TG_RW) run += g->reqs[a].hi - g->reqs[a].lo;
    }
    if (run > 0xFFFFFFFFull) return fail(TG_EINVAL, "task %u writes more than 2^32 elements", k);
  }
  InferResult res;
  tg_status is = tg_infer_dag_host(N, g->req_ptr.data(), g->reqs.data(), g->reqs.size(), g->space, res);
  if (is != TG_OK) return is;
  g->infer_ms = res.ms;
  g->succ_ptr = std::move(res.row_ptr);
  g->succ = std::move(res.col);
  // predecessor sets: transpose, rows ascending because j is visited in order
  g->dpred_ptr.assign((size_t)N + 1, 0);
  for (uint32_t k : g->succ) g->dpred_ptr[k + 1]++;
  for (uint32_t k = 0; k < N; ++k) g->dpred_ptr[k + 1] += g->dpred_ptr[k];
  g->dpred.assign(g->succ.size(), 0);
  {
    std::vector<uint64_t> fill(g->dpred_ptr.begin(), g->dpred_ptr.end() - 1);
    for (uint32_t j = 0; j < N; ++j)
      for (uint64_t x = g->succ_ptr[j]; x < g->succ_ptr[j + 1]; ++x) g->dpred[fill[g->succ[x]]++] = j;
  }
  g->level.assign(N, 0);
  for (uint32_t k = 0; k < N; ++k) {
    uint32_t lv = 0;
    for (uint64_t x = g->dpred_ptr[k]; x < g->dpred_ptr[k + 1]; ++x) lv = std::max(lv, g->level[g->dpred[x]] + 1);
    g->level[k] = lv;
  }
  g->xindeg.resize(N);
  for (uint32_t k = 0; k < N; ++k) g->xindeg[k] = (uint32_t)(g->dpred_ptr[k + 1] - g->dpred_ptr[k]);
  return TG_OK;
}

// ================================================================ C ABI

extern "C" {

const char* tg_status_str(tg_status s) {
  switch (s) {
    case TG_OK: return "TG_OK";
    case TG_EINVAL: return "TG_EINVAL";
    case TG_ENOMEM: return "TG_ENOMEM";
    case TG_EBUSY: return "TG_EBUSY";
    case TG_EDEVICE: return "TG_EDEVICE";
    case TG_ETIMEOUT: return "TG_ETIMEOUT";
    case TG_ESTATE: return "TG_ESTATE";
    default: return "TG_UNKNOWN";
  }
}

const char* tg_last_error(void) { return g_err.c_str(); }

const char* tg_version(void) { return "taskgraph-gfx950 0.1"; }

tg_status tg_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr)) return fail(TG_EINVAL, "alloc and free must both be set or both NULL");
  if (g_live.load() != 0) return fail(TG_EBUSY, "device buffers are alive; set the allocator first");
  g_alloc = alloc;
  g_free = free_;
  g_ctx = ctx;
  return TG_OK;
}

tg_status tg_graph_create(tg_graph* out, uint32_t mode, uint32_t payload_words, uint64_t index_space, uint64_t seed) {
  if (!out) return fail(TG_EINVAL, "out is NULL");
  *out = nullptr;
  if (mode == TG_EXPLICIT) {
    if (payload_words < 64 || payload_words > 65536 || (payload_words & (payload_words - 1)))
      return fail(TG_EINVAL, "payload_words must be a power of two in [64, 65536]");
  } else if (mode == TG_IMPLICIT) {
    if (index_space == 0 || index_space > (1ull << 36)) return fail(TG_EINVAL, "index_space must be in [1, 2^36]");
  } else {
    return fail(TG_EINVAL, "unknown mode %u", mode);
  }
  tg_graph g = new (std::nothrow) tg_graph_s();
  if (!g) return fail(TG_ENOMEM, "host allocation failed");
  g->mode = mode;
  g->n = mode == TG_EXPLICIT ? payload_words : 0;
  g->space = mode == TG_IMPLICIT ? index_space : 0;
  g->seed = seed;
  *out = g;
  return TG_OK;
}

tg_status tg_task_add_many(tg_graph g, uint32_t ntasks, const uint64_t* pred_ptr, const tg_event* preds,
                           const uint32_t* mix_rounds, uint32_t uniform_rounds, tg_event* first_event) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (g->mode != TG_EXPLICIT) return fail(TG_EINVAL, "graph is not in explicit mode");
  if (g->finalized) return fail(TG_EBUSY, "graph already finalised");
  if (ntasks && !pred_ptr) return fail(TG_EINVAL, "pred_ptr is NULL");
  const uint64_t N0 = g->N();
  if (N0 + ntasks >= 0xFFFFFFFFull) return fail(TG_EINVAL, "too many tasks");
  if (ntasks && pred_ptr[0] != 0) return fail(TG_EINVAL, "pred_ptr[0] must be 0");
  for (uint32_t i = 0; i < ntasks; ++i) {
    if (pred_ptr[i + 1] < pred_ptr[i]) return fail(TG_EINVAL, "pred_ptr not monotone at %u", i);
    for (uint64_t j = pred_ptr[i]; j < pred_ptr[i + 1]; ++j)
      if ((uint64_t)preds[j] >= N0 + i) return fail(TG_EINVAL, "task %llu names unknown event %u", (unsigned long long)(N0 + i), preds[j]);
  }
  const uint64_t E = ntasks ? pred_ptr[ntasks] : 0;
  const uint64_t base = g->preds.size();
  g->preds.insert(g->preds.end(), preds, preds + E);
  g->pred_ptr.reserve(g->pred_ptr.size() + ntasks);
  for (uint32_t i = 0; i < ntasks; ++i) g->pred_ptr.push_back(base + pred_ptr[i + 1]);
  for (uint32_t i = 0; i < ntasks; ++i) g->rounds.push_back(mix_rounds ? mix_rounds[i] : uniform_rounds);
  if (first_event) *first_event = (tg_event)N0;
  return TG_OK;
}

tg_status tg_task_add(tg_graph g, const tg_event* preds, uint32_t npreds, uint32_t mix_rounds, tg_event* out_event) {
  if (!out_event) return fail(TG_EINVAL, "out_event is NULL");
  if (npreds && !preds) return fail(TG_EINVAL, "preds is NULL");
  uint64_t ptr[2] = {0, npreds};
  return tg_task_add_many(g, 1, ptr, preds, nullptr, mix_rounds, out_event);
}

tg_status tg_task_add_regions_many(tg_graph g, uint32_t ntasks, const uint64_t* req_ptr, const tg_region_req* reqs,
                                   const uint32_t* mix_rounds, uint32_t uniform_rounds, tg_event* first_event) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (g->mode != TG_IMPLICIT) return fail(TG_EINVAL, "graph is not in implicit mode");
  if (g->finalized) return fail(TG_EBUSY, "graph already finalised");
  if (ntasks && !req_ptr) return fail(TG_EINVAL, "req_ptr is NULL");
  const uint64_t N0 = g->N();
  if (N0 + ntasks >= 0xFFFFFFFFull) return fail(TG_EINVAL, "too many tasks");
  if (ntasks && req_ptr[0] != 0) return fail(TG_EINVAL, "req_ptr[0] must be 0");
  for (uint32_t i = 0; i < ntasks; ++i) {
    if (req_ptr[i + 1] < req_ptr[i]) return fail(TG_EINVAL, "req_ptr not monotone at %u", i);
    for (uint64_t a = req_ptr[i]; a < req_ptr[i + 1]; ++a) {
      const tg_region_req& q = reqs[a];
      if (q.lo > q.hi || q.hi > g->space) return fail(TG_EINVAL, "task %llu: interval [%llu,%llu) outside index space",
                                                      (unsigned long long)(N0 + i), (unsigned long long)q.lo, (unsigned long long)q.hi);
      if (q.priv != TG_RO && q.priv != TG_RW) return fail(TG_EINVAL, "task %llu: bad privilege %u", (unsigned long long)(N0 + i), q.priv);
      for (uint64_t b = req_ptr[i]; b < req_ptr[i + 1]; ++b) {
        if (a == b) continue;
        const tg_region_req& r = reqs[b];
        if ((q.priv == TG_RW || r.priv == TG_RW) && q.lo < q.hi && r.lo < r.hi && q.lo < r.hi && r.lo < q.hi)
          return fail(TG_EINVAL, "task %llu: a read-write interval overlaps another interval of the same task",
                      (unsigned long long)(N0 + i));
      }
    }
  }
  const uint64_t M = ntasks ? req_ptr[ntasks] : 0;
  const uint64_t base = g->reqs.size();
  g->reqs.insert(g->reqs.end(), reqs, reqs + M);
  for (uint32_t i = 0; i < ntasks; ++i) g->req_ptr.push_back(base + req_ptr[i + 1]);
  for (uint32_t i = 0; i < ntasks; ++i) g->rounds.push_back(mix_rounds ? mix_rounds[i] : uniform_rounds);
  if (first_event) *first_event = (tg_event)N0;
  return TG_OK;
}

tg_status tg_task_add_regions(tg_graph g, const tg_region_req* reqs, uint32_t nreqs, uint32_t mix_rounds,
                              tg_event* out_event) {
  if (!out_event) return fail(TG_EINVAL, "out_event is NULL");
  if (nreqs && !reqs) return fail(TG_EINVAL, "reqs is NULL");
  uint64_t ptr[2] = {0, nreqs};
  return tg_task_add_regions_many(g, 1, ptr, reqs, nullptr, mix_rounds, out_event);
}

tg_status tg_graph_finalize(tg_graph g) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (g->finalized) return TG_OK;
  auto t0 = std::chrono::steady_clock::now();
  tg_status s = g->mode == TG_EXPLICIT ? finalize_explicit(g) : tg_finalize_implicit(g);
  if (s != TG_OK) return s;
  if ((s = build_blob(g)) != TG_OK) return s;
  g->finalized = true;
  g->compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() - g->infer_ms;
  return TG_OK;
}

static tg_status graph_execute(tg_graph g, const tg_exec_config* cfgp, void* stream, const LaunchConds* conds);

tg_status tg_graph_execute(tg_graph g, const tg_exec_config* cfgp, void* stream) {
  return graph_execute(g, cfgp, stream, nullptr);
}

static tg_status graph_execute(tg_graph g, const tg_exec_config* cfgp, void* stream, const LaunchConds* conds) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  // a new execution may follow an unwaited one on the same stream (stream
  // order serialises them); on another stream it must be waited for first
  if (g->inflight && (hipStream_t)stream != g->last_stream)
    return fail(TG_EBUSY, "previous execution on another stream not waited for");
  Config cfg = resolve(cfgp ? cfgp : (g->has_tuned ? &g->tuned : nullptr));
  tg_status s = check_config(cfg);
  if (s != TG_OK) return s;
  if (!g->solo || !same_layout(g->solo->cfg, cfg)) {
    if (g->inflight && (s = graph_wait(g)) != TG_OK) return s;
    drop_solo(g);
    std::vector<tg_graph> gs{g};
    if (!g->plans) g->plans = std::make_shared<PlanCache>();
    if ((s = build_layout(gs, cfg, g->solo, g->plans.get())) != TG_OK) return s;
  }
  hipStream_t st = (hipStream_t)stream;
  if ((s = ensure_events(g)) != TG_OK) return s;
  HIPCHK(hipEventRecord(g->ev0, st));
  std::vector<tg_graph> gs{g};
  const uint32_t slot = (uint32_t)(g->launches % tg_graph_s::kRing);
  if ((s = launch_layout(*g->solo, cfg, gs, st, g->evk, g->rk0[slot], g->rk1[slot], conds)) != TG_OK) return s;
  HIPCHK(hipEventRecord(g->ev1, st));
  g->launches++;
  g->inflight = true;
  g->last_stream = st;
  g->last_layout = g->solo.get();
  return TG_OK;
}

tg_status tg_graph_wait(tg_graph g) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  return graph_wait(g);
}

tg_status tg_graph_execute_after(tg_graph g, const tg_exec_config* cfg, void* stream, void* const* pre, uint32_t npre,
                                 void* post) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (npre && !pre) return fail(TG_EINVAL, "pre is NULL");
  hipStream_t st = (hipStream_t)stream;
  for (uint32_t i = 0; i < npre; ++i) {
    if (!pre[i]) return fail(TG_EINVAL, "pre[%u] is NULL", i);
    HIPCHK(hipStreamWaitEvent(st, (hipEvent_t)pre[i], 0));
  }
  tg_status s = tg_graph_execute(g, cfg, stream);
  if (s != TG_OK) return s;
  if (post) HIPCHK(hipEventRecord((hipEvent_t)post, st));
  return TG_OK;
}

// ---------------------------------------------------------------- flags

struct tg_flag_s {
  uint32_t* host = nullptr;  // one 128-byte line of pinned, coherent, mapped host memory
  uint32_t* dev = nullptr;   // the same word as the device addresses it
};

tg_status tg_flag_create(tg_flag* out) {
  if (!out) return fail(TG_EINVAL, "out is NULL");
  *out = nullptr;
  auto f = std::make_unique<tg_flag_s>();
  HIPCHK(hipHostMalloc((void**)&f->host, 128, hipHostMallocCoherent | hipHostMallocMapped));
  memset(f->host, 0, 128);
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, f->host, 0) != hipSuccess) {
    (void)hipHostFree(f->host);
    return fail(TG_EDEVICE, "hipHostGetDevicePointer failed for a flag");
  }
  f->dev = (uint32_t*)d;
  *out = f.release();
  return TG_OK;
}

tg_status tg_flag_destroy(tg_flag f) {
  if (!f) return TG_OK;
  if (f->host) (void)hipHostFree(f->host);
  delete f;
  return TG_OK;
}

tg_status tg_flag_set(tg_flag f, uint32_t value) {
  if (!f) return fail(TG_EINVAL, "flag is NULL");
  __atomic_store_n(f->host, value, __ATOMIC_SEQ_CST);
  return TG_OK;
}

tg_status tg_flag_read(tg_flag f, uint32_t* value) {
  if (!f || !value) return fail(TG_EINVAL, "NULL argument");
  *value = __atomic_load_n(f->host, __ATOMIC_ACQUIRE);
  return TG_OK;
}

tg_status tg_flag_wait(tg_flag f, uint32_t value, uint32_t timeout_ms) {
  if (!f) return fail(TG_EINVAL, "flag is NULL");
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spins = 0;; ++spins) {
    if (__atomic_load_n(f->host, __ATOMIC_ACQUIRE) >= value) return TG_OK;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms))
      return fail(TG_ETIMEOUT, "flag did not reach %u within %u ms", value, timeout_ms);
    if (spins > 64) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

tg_status tg_graph_execute_when(tg_graph g, const tg_exec_config* cfg, void* stream, const tg_flag* pre,
                                const uint32_t* pre_value, uint32_t npre, tg_flag post, uint32_t post_value) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (npre > tg::kMaxPreFlags) return fail(TG_EINVAL, "at most %u pre-condition flags, got %u", tg::kMaxPreFlags, npre);
  if (npre && (!pre || !pre_value)) return fail(TG_EINVAL, "pre or pre_value is NULL");
  LaunchConds c;
  for (uint32_t i = 0; i < npre; ++i) {
    if (!pre[i]) return fail(TG_EINVAL, "pre[%u] is NULL", i);
    c.pre.addr[i] = pre[i]->dev;
    c.pre.value[i] = pre_value[i];
  }
  c.pre.n = npre;
  if (post) {
    c.post = post->dev;
    c.post_value = post_value;
  }
  return graph_execute(g, cfg, stream, &c);
}

tg_status tg_graph_num_tasks(tg_graph g, uint64_t* n) {
  if (!g || !n) return fail(TG_EINVAL, "NULL argument");
  *n = g->N();
  return TG_OK;
}

tg_status tg_graph_num_edges(tg_graph g, uint64_t* e) {
  if (!g || !e) return fail(TG_EINVAL, "NULL argument");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  *e = g->succ.size();
  return TG_OK;
}

tg_status tg_graph_read_digests(tg_graph g, uint32_t* host_out, uint64_t n) {
  if (!g || !host_out) return fail(TG_EINVAL, "NULL argument");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  if (n != g->N()) return fail(TG_EINVAL, "n must equal the task count %u", g->N());
  if (g->released) {
    if (n) memcpy(host_out, g->host_digest.data(), n * 4);
    return TG_OK;
  }
  if (!g->digest.p) return fail(TG_ESTATE, "graph was never executed");
  tg_status s = graph_wait(g);
  if (s != TG_OK) return s;
  if (n) HIPCHK(hipMemcpy(host_out, g->digest.p, n * 4, hipMemcpyDeviceToHost));
  return TG_OK;
}

tg_status tg_graph_read_payload(tg_graph g, tg_event v, uint32_t* host_out, uint32_t n) {
  if (!g || !host_out) return fail(TG_EINVAL, "NULL argument");
  if (g->mode != TG_EXPLICIT) return fail(TG_EINVAL, "payloads exist in explicit mode only");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  if (v >= g->N() || n != g->n) return fail(TG_EINVAL, "bad event or payload size");
  if (!g->payload.p) return fail(TG_ESTATE, "graph was never executed");
  const uint32_t slot = g->slot_of.empty() ? v : g->slot_of[v];
  if (!g->slot_of.empty() && g->slot_last[slot] != v)
    return fail(TG_ESTATE, "the payload of task %u was released: its slot holds task %u's", v, g->slot_last[slot]);
  tg_status s = graph_wait(g);
  if (s != TG_OK) return s;
  HIPCHK(hipMemcpy(host_out, g->payload.as<uint32_t>() + (size_t)slot * g->n, (size_t)n * 4, hipMemcpyDeviceToHost));
  return TG_OK;
}

tg_status tg_graph_read_data(tg_graph g, uint32_t* host_out, uint64_t lo, uint64_t hi) {
  if (!g || !host_out) return fail(TG_EINVAL, "NULL argument");
  if (g->mode != TG_IMPLICIT) return fail(TG_EINVAL, "the shared array exists in implicit mode only");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  if (lo > hi || hi > g->space) return fail(TG_EINVAL, "range outside the index space");
  if (!g->data.p) return fail(TG_ESTATE, "the array is not on the device (never executed, or released)");
  tg_status s = graph_wait(g);
  if (s != TG_OK) return s;
  if (hi > lo) HIPCHK(hipMemcpy(host_out, g->data.as<uint32_t>() + lo, (hi - lo) * 4, hipMemcpyDeviceToHost));
  return TG_OK;
}

tg_status tg_graph_checksum(tg_graph g, uint64_t* out) {
  if (!g || !out) return fail(TG_EINVAL, "NULL argument");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  std::vector<uint32_t> d(g->N());
  tg_status s = tg_graph_read_digests(g, d.data(), d.size());
  if (s != TG_OK) return s;
  uint64_t c = 0;
  for (uint64_t v = 0; v < d.size(); ++v) c += (uint64_t)d[v] * (2ull * v + 1ull);
  *out = c;
  return TG_OK;
}

tg_status tg_graph_read_dag(tg_graph g, uint64_t* row_ptr, uint32_t* col, uint64_t cap_e, uint64_t* e) {
  if (!g || !row_ptr || !e) return fail(TG_EINVAL, "NULL argument");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  const bool apart = g->reduced || g->anti;
  const std::vector<uint64_t>& rp = apart ? g->full_succ_ptr : g->succ_ptr;
  const std::vector<uint32_t>& cl = apart ? g->full_succ : g->succ;
  *e = cl.size();
  memcpy(row_ptr, rp.data(), rp.size() * sizeof(uint64_t));
  if (cl.size() > cap_e) return fail(TG_ENOMEM, "col capacity %llu < %zu edges", (unsigned long long)cap_e, cl.size());
  if (!cl.empty()) {
    if (!col) return fail(TG_EINVAL, "col is NULL");
    memcpy(col, cl.data(), cl.size() * 4);
  }
  return TG_OK;
}

tg_status tg_graph_set_retention(tg_graph g, uint32_t mode) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (g->mode != TG_EXPLICIT) return fail(TG_EINVAL, "payload retention applies to explicit graphs");
  if (mode != TG_KEEP_ALL && mode != TG_KEEP_SINKS && mode != TG_KEEP_NONE)
    return fail(TG_EINVAL, "unknown retention mode %u", mode);
  if (g->finalized) return fail(TG_EBUSY, "set the retention before tg_graph_finalize");
  g->retain = mode;
  return TG_OK;
}

tg_status tg_graph_payload_slots(tg_graph g, uint32_t* slot_of, uint64_t* nslots, uint64_t* bytes) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  if (g->mode != TG_EXPLICIT) return fail(TG_EINVAL, "payloads exist in explicit mode only");
  if (slot_of)
    for (uint32_t v = 0; v < g->N(); ++v) slot_of[v] = g->slot_of.empty() ? v : g->slot_of[v];
  if (nslots) *nslots = g->nslots;
  if (bytes) *bytes = (uint64_t)g->nslots * g->n * 4ull;
  return TG_OK;
}

tg_status tg_graph_read_exec_dag(tg_graph g, uint64_t* row_ptr, uint32_t* col, uint64_t cap_e, uint64_t* e) {
  if (!g || !row_ptr || !e) return fail(TG_EINVAL, "NULL argument");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  *e = g->succ.size();
  memcpy(row_ptr, g->succ_ptr.data(), g->succ_ptr.size() * sizeof(uint64_t));
  if (g->succ.size() > cap_e) return fail(TG_ENOMEM, "col capacity %llu < %zu edges", (unsigned long long)cap_e, g->succ.size());
  if (!g->succ.empty()) {
    if (!col) return fail(TG_EINVAL, "col is NULL");
    memcpy(col, g->succ.data(), g->succ.size() * 4);
  }
  return TG_OK;
}

// Last-user dependences of an implicit program (Section 5: dependences only
// have to order conflicting tasks as program order does).  Walks the tasks in
// program order over a map of element runs that share one history: the last
// task that wrote the run and the tasks that read it since.  A task that
// reads a run depends on its last writer; a task that writes it depends on
// the last writer and every reader since, and becomes the run's only user.
// Every edge joins two conflicting tasks, and every conflicting pair j < k is
// joined by a path through the writers of a shared element between them, so
// the order imposed is the conflict DAG's.  Out-edge CSR, rows ascending.
static void last_user_dag(uint32_t N, const uint64_t* req_ptr, const tg_region_req* reqs,
                          std::vector<uint64_t>& rp, std::vector<uint32_t>& cl) {
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  struct Run {
    uint64_t hi;
    uint32_t writer;
    std::vector<uint32_t> readers;  // ascending, no repeats
  };
  std::map<uint64_t, Run> runs;  // key: first element of the run
  runs.emplace(0, Run{UINT64_MAX, kNone, {}});
  auto split = [&](uint64_t x) {  // make x the start of a run
    auto it = std::prev(runs.upper_bound(x));
    if (it->first == x) return;
    Run tail{it->second.hi, it->second.writer, it->second.readers};
    it->second.hi = x;
    runs.emplace_hint(std::next(it), x, std::move(tail));
  };
  std::vector<uint64_t> pp(N + 1, 0);
  std::vector<uint32_t> pr, preds;
  for (uint32_t k = 0; k < N; ++k) {
    preds.clear();
    for (uint64_t a = req_ptr[k]; a < req_ptr[k + 1]; ++a) {
      const tg_region_req& q = reqs[a];
      if (q.lo >= q.hi) continue;
      split(q.lo);
      if (q.hi != UINT64_MAX) split(q.hi);
      auto it = runs.find(q.lo);
      if (q.priv == TG_RW) {
        for (auto jt = it; jt != runs.end() && jt->first < q.hi; ++jt) {
          if (jt->second.writer != kNone) preds.push_back(jt->second.writer);
          preds.insert(preds.end(), jt->second.readers.begin(), jt->second.readers.end());
        }
        // the written interval becomes one run whose only user is k
        const uint64_t hi = q.hi;
        auto end = runs.lower_bound(hi);
        runs.erase(it, end);
        runs.emplace(q.lo, Run{hi, k, {}});
      } else {
        for (auto jt = it; jt != runs.end() && jt->first < q.hi; ++jt) {
          if (jt->second.writer != kNone) preds.push_back(jt->second.writer);
          std::vector<uint32_t>& rd = jt->second.readers;
          if (rd.empty() || rd.back() != k) rd.push_back(k);
        }
      }
    }
    std::sort(preds.begin(), preds.end());
    preds.erase(std::unique(preds.begin(), preds.end()), preds.end());
    while (!preds.empty() && preds.back() == k) preds.pop_back();  // its own earlier interval
    pr.insert(pr.end(), preds.begin(), preds.end());
    pp[k + 1] = pr.size();
  }
  // predecessor rows -> successor rows (ascending: k is visited in order)
  rp.assign(N + 1, 0);
  for (uint32_t j : pr) rp[j + 1]++;
  for (uint32_t j = 0; j < N; ++j) rp[j + 1] += rp[j];
  cl.resize(pr.size());
  std::vector<uint64_t> fill(rp.begin(), rp.end() - 1);
  for (uint32_t k = 0; k < N; ++k)
    for (uint64_t x = pp[k]; x < pp[k + 1]; ++x) cl[fill[pr[x]]++] = k;
}

tg_status tg_last_user_dag(uint32_t n, const uint64_t* req_ptr, const tg_region_req* reqs, uint64_t* out_row_ptr,
                           uint32_t* out_col, uint64_t cap_e, uint64_t* out_e) {
  if (!req_ptr || !out_row_ptr || !out_e) return fail(TG_EINVAL, "NULL argument");
  if (req_ptr[0] != 0) return fail(TG_EINVAL, "req_ptr[0] = %llu, not 0", (unsigned long long)req_ptr[0]);
  for (uint32_t k = 0; k < n; ++k)
    if (req_ptr[k + 1] < req_ptr[k]) return fail(TG_EINVAL, "req_ptr not ascending at %u", k);
  if (req_ptr[n] && !reqs) return fail(TG_EINVAL, "reqs is NULL");
  for (uint64_t a = 0; a < req_ptr[n]; ++a) {
    if (reqs[a].lo > reqs[a].hi) return fail(TG_EINVAL, "requirement %llu: lo > hi", (unsigned long long)a);
    if (reqs[a].priv != TG_RO && reqs[a].priv != TG_RW)
      return fail(TG_EINVAL, "requirement %llu: unknown privilege %u", (unsigned long long)a, reqs[a].priv);
  }
  std::vector<uint64_t> rp;
  std::vector<uint32_t> cl;
  last_user_dag(n, req_ptr, reqs, rp, cl);
  *out_e = cl.size();
  if (cl.size() > cap_e) return fail(TG_ENOMEM, "col capacity %llu < %zu edges", (unsigned long long)cap_e, cl.size());
  memcpy(out_row_ptr, rp.data(), (n + 1) * sizeof(uint64_t));
  if (!cl.empty()) {
    if (!out_col) return fail(TG_EINVAL, "out_col is NULL");
    memcpy(out_col, cl.data(), cl.size() * 4);
  }
  return TG_OK;
}

tg_status tg_graph_reduce_edges(tg_graph g, uint64_t* removed) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  if (g->mode != TG_IMPLICIT)
    return fail(TG_EINVAL, "only implicit graphs: an explicit task's predecessors are its inputs");
  tg_status s = graph_wait(g);
  if (s != TG_OK) return s;
  if (g->reduced) {
    if (removed) *removed = g->full_succ.size() - g->succ.size();
    return TG_OK;
  }
  const uint32_t N = g->N();
  // the last-user DAG orders the tasks as the inferred DAG does with a few
  // edges per task; the two-hop pass then drops what paths imply
  std::vector<uint64_t> lrp;
  std::vector<uint32_t> lcl;
  last_user_dag(N, g->req_ptr.data(), g->reqs.data(), lrp, lcl);
  std::vector<uint64_t> rp(N + 1);
  std::vector<uint32_t> cl(lcl.size());
  uint64_t e = 0;
  if ((s = tg_reduce_dag(N, lrp.data(), lcl.data(), rp.data(), cl.data(), &e)) != TG_OK) return s;
  cl.resize(e);
  g->full_succ_ptr.swap(g->succ_ptr);
  g->full_succ.swap(g->succ);
  g->succ_ptr.swap(rp);
  g->succ.swap(cl);
  // predecessor lists of the reduced edges (ascending)
  std::vector<uint64_t> pp(N + 1, 0);
  for (uint32_t x : g->succ) pp[x + 1]++;
  for (uint32_t k = 0; k < N; ++k) pp[k + 1] += pp[k];
  std::vector<uint32_t> pr(g->succ.size());
  {
    std::vector<uint64_t> fill(pp.begin(), pp.end() - 1);
    for (uint32_t j = 0; j < N; ++j)
      for (uint64_t a = g->succ_ptr[j]; a < g->succ_ptr[j + 1]; ++a) pr[fill[g->succ[a]]++] = j;
  }
  g->dpred_ptr.swap(pp);
  g->dpred.swap(pr);
  for (uint32_t k = 0; k < N; ++k) g->xindeg[k] = (uint32_t)(g->dpred_ptr[k + 1] - g->dpred_ptr[k]);
  if ((s = build_blob(g)) != TG_OK) return s;
  g->reduced = true;
  // layouts and schedules were built on the full edge set
  drop_solo(g);
  g->plans.reset();
  g->has_tuned = false;
  if (removed) *removed = g->full_succ.size() - g->succ.size();
  return TG_OK;
}

// Two-hop reduction of a DAG whose vertex ids are a topological order: the
// edge j -> k is dropped when some i has edges j -> i and i -> k.  Every
// dropped edge is implied by a path of the input, so reachability is
// unchanged (all edges of the transitive reduction are kept).
tg_status tg_reduce_dag(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, uint64_t* out_row_ptr,
                        uint32_t* out_col, uint64_t* out_e) {
  if (!row_ptr || !out_row_ptr || !out_e) return fail(TG_EINVAL, "NULL argument");
  const uint64_t E = row_ptr[n];
  if (E && (!col || !out_col)) return fail(TG_EINVAL, "NULL edge array");
  for (uint32_t j = 0; j < n; ++j) {
    if (row_ptr[j + 1] < row_ptr[j]) return fail(TG_EINVAL, "row_ptr not ascending at %u", j);
    for (uint64_t a = row_ptr[j]; a < row_ptr[j + 1]; ++a)
      if (col[a] <= j || col[a] >= n) return fail(TG_EINVAL, "edge %u -> %u does not go forward", j, col[a]);
  }
  // predecessor lists
  std::vector<uint64_t> pp(n + 1, 0);
  for (uint64_t a = 0; a < E; ++a) pp[col[a] + 1]++;
  for (uint32_t k = 0; k < n; ++k) pp[k + 1] += pp[k];
  std::vector<uint32_t> pr(E);
  {
    std::vector<uint64_t> fill(pp.begin(), pp.end() - 1);
    for (uint32_t j = 0; j < n; ++j)
      for (uint64_t a = row_ptr[j]; a < row_ptr[j + 1]; ++a) pr[fill[col[a]]++] = j;
  }
  // keep[x]: predecessor entry x (edge pr[x] -> k) survives
  std::vector<uint8_t> keep(E, 1);
  auto work = [&](uint32_t k0, uint32_t k1) {
    std::vector<uint32_t> stamp(n, 0xFFFFFFFFu);
    std::vector<uint64_t> where(n, 0);
    for (uint32_t k = k0; k < k1; ++k) {
      for (uint64_t x = pp[k]; x < pp[k + 1]; ++x) {
        stamp[pr[x]] = k;
        where[pr[x]] = x;
      }
      for (uint64_t x = pp[k]; x < pp[k + 1]; ++x) {
        const uint32_t i = pr[x];
        for (uint64_t y = pp[i]; y < pp[i + 1]; ++y)
          if (stamp[pr[y]] == k) keep[where[pr[y]]] = 0;
      }
    }
  };
  const uint32_t nth = n >= 4096 ? std::max(1u, std::min(8u, std::thread::hardware_concurrency())) : 1u;
  if (nth <= 1) {
    work(0, n);
  } else {
    std::vector<std::thread> pool;
    for (uint32_t t = 0; t < nth; ++t)
      pool.emplace_back(work, (uint32_t)((uint64_t)n * t / nth), (uint32_t)((uint64_t)n * (t + 1) / nth));
    for (auto& th : pool) th.join();
  }
  // reduced successor CSR (rows ascending because predecessors are visited
  // in ascending k)
  std::fill(out_row_ptr, out_row_ptr + n + 1, 0);
  for (uint32_t k = 0; k < n; ++k)
    for (uint64_t x = pp[k]; x < pp[k + 1]; ++x)
      if (keep[x]) out_row_ptr[pr[x] + 1]++;
  for (uint32_t j = 0; j < n; ++j) out_row_ptr[j + 1] += out_row_ptr[j];
  std::vector<uint64_t> fill(out_row_ptr, out_row_ptr + n);
  for (uint32_t k = 0; k < n; ++k)
    for (uint64_t x = pp[k]; x < pp[k + 1]; ++x)
      if (keep[x]) out_col[fill[pr[x]]++] = k;
  *out_e = out_row_ptr[n];
  return TG_OK;
}

tg_status tg_graph_timings(tg_graph g, double* compile_ms, double* infer_ms, double* exec_ms) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (compile_ms) *compile_ms = g->compile_ms;
  if (infer_ms) *infer_ms = g->infer_ms;
  if (exec_ms) *exec_ms = g->exec_ms;
  return TG_OK;
}

tg_status tg_graph_kernel_ms(tg_graph g, double* kernel_ms) {
  if (!g || !kernel_ms) return fail(TG_EINVAL, "NULL argument");
  *kernel_ms = g->kernel_ms;
  return TG_OK;
}

tg_status tg_graph_kernel_times(tg_graph g, double* ms_out, uint32_t n, uint32_t* got) {
  if (!g || !ms_out || !got) return fail(TG_EINVAL, "NULL argument");
  tg_status s = graph_wait(g);
  if (s != TG_OK) return s;
  uint64_t have = g->launches < tg_graph_s::kRing ? g->launches : tg_graph_s::kRing;
  if (n < have) have = n;
  for (uint64_t i = 0; i < have; ++i) {
    const uint64_t k = g->launches - have + i;
    const uint32_t slot = (uint32_t)(k % tg_graph_s::kRing);
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, g->rk0[slot], g->rk1[slot]));
    ms_out[i] = ms;
  }
  *got = (uint32_t)have;
  return TG_OK;
}

tg_status tg_graph_set_rounds(tg_graph g, uint32_t uniform_rounds) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  tg_status s = graph_wait(g);
  if (s != TG_OK) return s;
  std::fill(g->rounds.begin(), g->rounds.end(), uniform_rounds);
  if (g->finalized) {
    std::fill(g->blob.begin() + g->bo.rounds, g->blob.begin() + g->bo.rounds + g->N(), uniform_rounds);
    g->blob_gen++;
  }
  if (g->solo) {
    Layout& L = *g->solo;
    for (auto& r : L.rec_host) r.rounds = uniform_rounds;
    if (!L.rec_host.empty())
      HIPCHK(hipMemcpy(L.rec.p, L.rec_host.data(), L.rec_host.size() * sizeof(TaskRec), hipMemcpyHostToDevice));
  }
  return null_stream_fence();
}

// Median number of tasks per dependence level over levels 1.. of a set of
// graphs (levels of different graphs with the same index counted together).
// A level-ordered layout with this many workers gives every worker one task
// per level, mostly of the same column, so it waits on its own last task.
static uint32_t typical_level_width(const std::vector<tg_graph>& gs) {
  std::vector<uint32_t> width;
  for (auto g : gs)
    for (uint32_t lv : g->level) {
      if (lv >= width.size()) width.resize(lv + 1, 0);
      width[lv]++;
    }
  if (width.size() < 2) return width.empty() ? 0 : width[0];
  std::vector<uint32_t> w(width.begin() + 1, width.end());
  std::nth_element(w.begin(), w.begin() + w.size() / 2, w.end());
  return w[w.size() / 2];
}

tg_status tg_graph_autotune(tg_graph g, uint32_t reps, tg_exec_config* best, double* best_ms) {
  if (!g || !best) return fail(TG_EINVAL, "NULL argument");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  if (reps == 0) reps = 2;
  tg_status s = graph_wait(g);
  if (s != TG_OK) return s;
  // candidate launch configurations
  std::vector<tg_exec_config> cand;
  DevInfo di;
  if ((s = device_info(di)) != TG_OK) return s;
  const uint32_t cus = (uint32_t)di.cus;
  uint32_t rw = 0, rg2 = 0, rg4 = 0, rg8 = 0, rg16 = 0;
  if ((s = resident_workers(TG_MAP_WORKGROUP, 16, &rg16)) != TG_OK) return s;
  if ((s = resident_workers(TG_MAP_WORKGROUP, 8, &rg8)) != TG_OK) return s;
  if ((s = resident_workers(TG_MAP_WAVE, 4, &rw)) != TG_OK) return s;
  if ((s = resident_workers(TG_MAP_WORKGROUP, 2, &rg2)) != TG_OK) return s;
  if ((s = resident_workers(TG_MAP_WORKGROUP, 4, &rg4)) != TG_OK) return s;
  auto mk = [](uint32_t m, uint32_t w, uint32_t ww, uint32_t nt) {
    tg_exec_config c;
    memset(&c, 0, sizeof(c));
    c.mapping = m;
    c.workers = w;
    c.wg_waves = ww;
    c.notify = nt;
    return c;
  };
  for (uint32_t sch : {TG_SCHED_LIST, TG_SCHED_LEVEL, TG_SCHED_SPREAD, TG_SCHED_COLUMN, TG_SCHED_BALANCED}) {
    std::vector<tg_exec_config> shapes;
    for (uint32_t w : {rw, rw / 4, rw / 8})
      if (w) shapes.push_back(mk(TG_MAP_WAVE, w, 0, 0));
    shapes.push_back(mk(TG_MAP_WORKGROUP, rg2, 2, 0));
    shapes.push_back(mk(TG_MAP_WORKGROUP, rg4, 4, 0));
    // one large workgroup per CU: for graphs with few, large tasks
    for (uint32_t ww : {8u, 16u}) shapes.push_back(mk(TG_MAP_WORKGROUP, cus, ww, 0));
    // one worker per task of a typical level
    const uint32_t lw = typical_level_width(std::vector<tg_graph>{g});
    if (lw >= 64 && lw <= rw && lw != rw && lw != rw / 4 && lw != rw / 8) shapes.push_back(mk(TG_MAP_WAVE, lw, 0, 0));
    // gangs of workgroups on several CUs per task, for large tasks: every
    // resident gang, or three quarters of them (which gangs share a CU, and
    // so how evenly the busy members of a level spread over the CUs, depends
    // on the gang count: measured up to 6 % apart on a 64-wide wavefront)
    const uint32_t gshape[][3] = {{16, 4, rg16}, {8, 4, rg8}, {8, 8, rg8}, {4, 16, rg4}};
    for (const auto& gsh : gshape)
      for (uint32_t n : {gsh[2] / gsh[1], gsh[2] / gsh[1] * 3 / 4})
        if (n) {
          shapes.push_back(mk(TG_MAP_GANG, n, gsh[0], 0));
          shapes.back().gang = gsh[1];
        }
    for (auto c : shapes) {
      c.schedule = sch;
      cand.push_back(c);
    }
  }
  cand.push_back(mk(TG_MAP_WAVE, rw, 0, 1));
  // ready-queue dispatch, unless the DAG is dense (an inferred conflict DAG
  // links each task to every later task of its region: every completion
  // then pays a ballot and a push round over tens of out-edges, and the
  // queue has been measured several times slower than the lists there)
  if (g->succ.size() <= 16ull * g->N())
    for (uint32_t tile : {1u, 4u}) {
      for (uint32_t w : {rw, rw / 2}) {
        tg_exec_config c = mk(TG_MAP_WAVE, w, 0, 0);
        c.dispatch = TG_DISPATCH_QUEUE;
        c.tile = tile;
        cand.push_back(c);
      }
      tg_exec_config c = mk(TG_MAP_WORKGROUP, rg4, 4, 0);
      c.dispatch = TG_DISPATCH_QUEUE;
      c.tile = tile;
      cand.push_back(c);
    }
  double best_t = 1e300;
  tg_exec_config best_c = cand[0];
  for (const auto& c : cand) {
    double tot = 0;
    uint32_t timed = 0;
    for (uint32_t r = 0; r <= reps; ++r) {  // first run warms up
      if ((s = tg_graph_execute(g, &c, nullptr)) != TG_OK) return s;
      if ((s = graph_wait(g)) != TG_OK) return s;
      // a candidate whose warm-up took several times the best mean so far
      // cannot win: its timed runs are skipped
      if (r == 0 && g->kernel_ms > 4.0 * best_t) break;
      if (r) {
        tot += g->kernel_ms;
        ++timed;
      }
    }
    if (!timed) continue;
    const double mean = tot / timed;
    if (mean < best_t) {
      best_t = mean;
      best_c = c;
    }
  }
  g->tuned = best_c;
  g->has_tuned = true;
  *best = best_c;
  if (best_ms) *best_ms = best_t;
  return TG_OK;
}

tg_status tg_graph_destroy(tg_graph g) {
  if (!g) return TG_OK;
  (void)graph_wait(g);
  drop_solo(g);
  if (g->ev0) (void)hipEventDestroy(g->ev0);
  if (g->ev1) (void)hipEventDestroy(g->ev1);
  if (g->evk) (void)hipEventDestroy(g->evk);
  for (uint32_t i = 0; i < tg_graph_s::kRing; ++i) {
    if (g->rk0[i]) (void)hipEventDestroy(g->rk0[i]);
    if (g->rk1[i]) (void)hipEventDestroy(g->rk1[i]);
  }
  delete g;
  return TG_OK;
}

// ---------------------------------------------------------------- batches

tg_status tg_batch_create(tg_batch* out, const tg_graph* graphs, uint32_t n, const tg_exec_config* cfgp) {
  if (!out || (n && !graphs)) return fail(TG_EINVAL, "NULL argument");
  *out = nullptr;
  std::vector<tg_graph> gs(graphs, graphs + n);
  for (auto g : gs) {
    if (!g) return fail(TG_EINVAL, "NULL graph in batch");
    if (!g->finalized) return fail(TG_ESTATE, "every graph of a batch must be finalised");
  }
  Config cfg = resolve(cfgp);
  auto b = std::make_unique<tg_batch_s>();
  b->graphs = gs;
  b->plans = std::make_shared<PlanCache>();
  tg_status s = build_layout(gs, cfg, b->lay, b->plans.get());
  if (s != TG_OK) return s;
  for (auto g : gs) b->gens.push_back(g->dev_gen);
  HIPCHK(hipEventCreate(&b->ev0));
  HIPCHK(hipEventCreate(&b->ev1));
  for (uint32_t i = 0; i < tg_batch_s::kRing; ++i) {
    HIPCHK(hipEventCreate(&b->rk0[i]));
    HIPCHK(hipEventCreate(&b->rk1[i]));
  }
  *out = b.release();
  return TG_OK;
}

tg_status tg_batch_execute(tg_batch b, void* stream) {
  if (!b) return fail(TG_EINVAL, "batch is NULL");
  if (b->inflight && (hipStream_t)stream != b->last_stream)
    return fail(TG_EBUSY, "previous execution on another stream not waited for");
  if (!b->inflight)
    for (auto g : b->graphs) {
      tg_status s = graph_wait(g);
      if (s != TG_OK) return s;
    }
  // the layout holds the graphs' device addresses: refuse to run if any
  // graph's buffers were released or reallocated since
  for (size_t i = 0; i < b->graphs.size(); ++i)
    if (b->graphs[i]->dev_gen != b->gens[i] || b->graphs[i]->released)
      return fail(TG_ESTATE, "graph %zu of the batch lost its device buffers; create the batch again", i);
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipEventRecord(b->ev0, st));
  const uint32_t slot = (uint32_t)(b->launches % tg_batch_s::kRing);
  tg_status s = launch_layout(*b->lay, b->lay->cfg, b->graphs, st, nullptr, b->rk0[slot], b->rk1[slot]);
  if (s != TG_OK) return s;
  HIPCHK(hipEventRecord(b->ev1, st));
  b->launches++;
  b->inflight = true;
  b->last_stream = st;
  return TG_OK;
}

tg_status tg_batch_wait(tg_batch b) {
  if (!b) return fail(TG_EINVAL, "batch is NULL");
  if (!b->inflight) return TG_OK;
  b->inflight = false;
  HIPCHK(hipEventSynchronize(b->ev1));
  return check_abort(b->lay.get());
}

tg_status tg_batch_time_ms(tg_batch b, double* ms) {
  if (!b || !ms) return fail(TG_EINVAL, "NULL argument");
  float f = 0;
  HIPCHK(hipEventElapsedTime(&f, b->ev0, b->ev1));
  *ms = f;
  return TG_OK;
}

tg_status tg_batch_kernel_times(tg_batch b, double* ms_out, uint32_t n, uint32_t* got) {
  if (!b || !ms_out || !got) return fail(TG_EINVAL, "NULL argument");
  tg_status s = tg_batch_wait(b);
  if (s != TG_OK) return s;
  uint64_t have = b->launches < tg_batch_s::kRing ? b->launches : tg_batch_s::kRing;
  if (n < have) have = n;
  for (uint64_t i = 0; i < have; ++i) {
    const uint32_t slot = (uint32_t)((b->launches - have + i) % tg_batch_s::kRing);
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, b->rk0[slot], b->rk1[slot]));
    ms_out[i] = ms;
  }
  *got = (uint32_t)have;
  return TG_OK;
}

tg_status tg_batch_set_rounds(tg_batch b, uint32_t uniform_rounds) {
  if (!b) return fail(TG_EINVAL, "batch is NULL");
  tg_status s = tg_batch_wait(b);
  if (s != TG_OK) return s;
  for (auto g : b->graphs) std::fill(g->rounds.begin(), g->rounds.end(), uniform_rounds);
  Layout& L = *b->lay;
  for (auto& r : L.rec_host) r.rounds = uniform_rounds;
  if (!L.rec_host.empty())
    HIPCHK(hipMemcpy(L.rec.p, L.rec_host.data(), L.rec_host.size() * sizeof(TaskRec), hipMemcpyHostToDevice));
  return null_stream_fence();
}

tg_status tg_batch_signalled_edges(tg_batch b, uint64_t* edges) {
  if (!b || !edges) return fail(TG_EINVAL, "NULL argument");
  *edges = b->lay->signalled;
  return TG_OK;
}

tg_status tg_batch_info(tg_batch b, tg_exec_config* cfg, uint64_t* tasks, double* plan_ms, double* build_ms) {
  if (!b) return fail(TG_EINVAL, "batch is NULL");
  if (plan_ms) *plan_ms = b->lay->plan_ms;
  if (build_ms) *build_ms = b->lay->build_ms;
  if (cfg) {
    memset(cfg, 0, sizeof(*cfg));
    const Config& c = b->lay->cfg;
    cfg->mapping = c.mapping;
    cfg->workers = b->lay->nworkers;
    cfg->window = c.window;
    cfg->wg_waves = c.wg_waves;
    cfg->watchdog_ms = c.watchdog_ms;
    cfg->notify = c.notify;
    cfg->idle_sleep = c.idle_sleep;
    cfg->schedule = c.schedule;
    cfg->gang = c.mapping == TG_MAP_GANG ? c.gang : 0;
    cfg->dispatch = c.dispatch;
    cfg->tile = c.dispatch == TG_DISPATCH_QUEUE ? c.tile : 0;
    cfg->shards = c.dispatch == TG_DISPATCH_QUEUE ? c.shards : 0;
  }
  if (tasks) *tasks = b->lay->npos;
  return TG_OK;
}

// Autotuner for a batch: rebuild the layout for each candidate launch shape,
// time reps executions, keep the fastest.
tg_status tg_batch_autotune(tg_batch b, uint32_t reps, tg_exec_config* best, double* best_ms) {
  if (!b || !best) return fail(TG_EINVAL, "NULL argument");
  if (reps == 0) reps = 2;
  tg_status s = tg_batch_wait(b);
  if (s != TG_OK) return s;
  uint32_t rw = 0, rg2 = 0, rg4 = 0;
  if ((s = resident_workers(TG_MAP_WAVE, 4, &rw)) != TG_OK) return s;
  if ((s = resident_workers(TG_MAP_WORKGROUP, 2, &rg2)) != TG_OK) return s;
  if ((s = resident_workers(TG_MAP_WORKGROUP, 4, &rg4)) != TG_OK) return s;
  if (!b->plans) b->plans = std::make_shared<PlanCache>();
  std::vector<Config> cand;
  auto mk = [](uint32_t m, uint32_t w, uint32_t ww, uint32_t nt) {
    Config c;
    c.mapping = m;
    c.workers = w;
    if (ww) c.wg_waves = ww;
    c.notify = nt;
    return c;
  };
  for (uint32_t sch : {TG_SCHED_LIST, TG_SCHED_LEVEL, TG_SCHED_SPREAD, TG_SCHED_COLUMN, TG_SCHED_BALANCED}) {
    std::vector<Config> shapes;
    for (uint32_t w : {rw, rw / 4})
      if (w) shapes.push_back(mk(TG_MAP_WAVE, w, 0, 0));
    // one worker per task of a typical level
    const uint32_t lw = typical_level_width(b->graphs);
    if (lw >= 64 && lw <= rw && lw != rw && lw != rw / 4) shapes.push_back(mk(TG_MAP_WAVE, lw, 0, 0));
    shapes.push_back(mk(TG_MAP_WORKGROUP, rg2, 2, 0));
    shapes.push_back(mk(TG_MAP_WORKGROUP, rg4, 4, 0));
    for (auto c : shapes) {
      c.schedule = sch;
      cand.push_back(c);
    }
  }
  cand.push_back(mk(TG_MAP_WAVE, rw, 0, 1));
  // ready-queue dispatch
  for (uint32_t tile : {1u, 4u}) {
    for (uint32_t w : {rw, rw / 2}) {
      Config c = mk(TG_MAP_WAVE, w, 0, 0);
      c.dispatch = TG_DISPATCH_QUEUE;
      c.tile = tile;
      cand.push_back(c);
    }
    Config c = mk(TG_MAP_WORKGROUP, rg4, 4, 0);
    c.dispatch = TG_DISPATCH_QUEUE;
    c.tile = tile;
    cand.push_back(c);
  }
  double best_t = 1e300;
  Config best_c = cand[0];
  for (const auto& c : cand) {
    b->lay.reset();
    if ((s = build_layout(b->graphs, c, b->lay, b->plans.get())) != TG_OK) return s;
    double tot = 0;
    uint32_t timed = 0;
    for (uint32_t r = 0; r <= reps; ++r) {
      if ((s = tg_batch_execute(b, nullptr)) != TG_OK) return s;
      if ((s = tg_batch_wait(b)) != TG_OK) return s;
      float ms = 0;
      const uint32_t slot = (uint32_t)((b->launches - 1) % tg_batch_s::kRing);
      HIPCHK(hipEventElapsedTime(&ms, b->rk0[slot], b->rk1[slot]));
      if (r == 0 && ms > 4.0 * best_t) break;  // cannot win: skip the timed runs
      if (r) {
        tot += ms;
        ++timed;
      }
    }
    if (timed && tot / timed < best_t) {
      best_t = tot / timed;
      best_c = c;
    }
  }
  b->lay.reset();
  if ((s = build_layout(b->graphs, best_c, b->lay, b->plans.get())) != TG_OK) return s;
  b->gens.clear();
  for (auto g : b->graphs) b->gens.push_back(g->dev_gen);
  if ((s = tg_batch_info(b, best, nullptr, nullptr, nullptr)) != TG_OK) return s;
  if (best_ms) *best_ms = best_t;
  return TG_OK;
}

tg_status tg_batch_destroy(tg_batch b) {
  if (!b) return TG_OK;
  (void)tg_batch_wait(b);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  for (uint32_t i = 0; i < tg_batch_s::kRing; ++i) {
    if (b->rk0[i]) (void)hipEventDestroy(b->rk0[i]);
    if (b->rk1[i]) (void)hipEventDestroy(b->rk1[i]);
  }
  delete b;
  return TG_OK;
}

// ------------------------------------------------------------ comparators

tg_status tg_exec_occupancy(uint32_t mapping, uint32_t wg_waves, uint32_t* blocks_per_cu, uint32_t* cus,
                            uint32_t* resident) {
  if (!blocks_per_cu || !cus) return fail(TG_EINVAL, "NULL argument");
  if (mapping != TG_MAP_WAVE && mapping != TG_MAP_WORKGROUP) return fail(TG_EINVAL, "mapping must be 1 or 2");
  if (wg_waves < 1 || wg_waves > 16) return fail(TG_EINVAL, "wg_waves must be in [1, 16]");
  DevInfo di;
  tg_status s = device_info(di);
  if (s != TG_OK) return s;
  int b = tg::exec_blocks_per_cu(mapping, wg_waves);
  if (b <= 0) return fail(TG_EDEVICE, "occupancy query failed");
  *blocks_per_cu = (uint32_t)b;
  *cus = (uint32_t)di.cus;
  if (resident) return resident_workers(mapping, wg_waves, resident);
  return TG_OK;
}

tg_status tg_graph_debug_times(tg_graph g, uint64_t* task_times, uint64_t* worker_stamps, uint32_t nworkers) {
  if (!g || !task_times) return fail(TG_EINVAL, "NULL argument");
  if (!g->solo || !g->solo->tstamp.p) return fail(TG_ESTATE, "no diagnostic launch");
  Layout& L = *g->solo;
  (void)hipDeviceSynchronize();
  std::vector<uint64_t> t((size_t)L.npos * 2);
  HIPCHK(hipMemcpy(t.data(), L.tstamp.p, t.size() * 8, hipMemcpyDeviceToHost));
  for (uint32_t v = 0; v < g->N(); ++v) {
    task_times[2 * v] = t[2 * L.pos_of[0][v]];
    task_times[2 * v + 1] = t[2 * L.pos_of[0][v] + 1];
  }
  if (worker_stamps) {
    if (nworkers != L.nworkers) return fail(TG_EINVAL, "nworkers must be %u", L.nworkers);
    HIPCHK(hipMemcpy(worker_stamps, L.wstamp.p, (size_t)L.nworkers * 32, hipMemcpyDeviceToHost));
  }
  return TG_OK;
}

tg_status tg_graph_debug_state(tg_graph g, uint32_t* pending, uint32_t* execs, uint32_t* owner, uint32_t* entry,
                               uint32_t* wprog, uint32_t nworkers) {
  if (!g || !pending || !execs || !owner || !entry) return fail(TG_EINVAL, "NULL argument");
  if (!g->solo) return fail(TG_ESTATE, "graph was never executed");
  Layout& L = *g->solo;
  if (!L.execs.p) return fail(TG_ESTATE, "last launch was not a diagnostic launch");
  (void)hipStreamSynchronize(nullptr);
  (void)hipDeviceSynchronize();
  const uint32_t N = g->N();
  std::vector<uint32_t> c(L.npos), x(L.npos), wb(L.nworkers + 1);
  HIPCHK(hipMemcpy(c.data(), L.cnt.p, (size_t)L.npos * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(x.data(), L.execs.p, (size_t)L.npos * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(wb.data(), L.wbase.p, wb.size() * 4, hipMemcpyDeviceToHost));
  for (uint32_t v = 0; v < N; ++v) {
    const uint32_t pos = L.pos_of[0][v];
    pending[v] = c[pos] & tg::kPendingMask;
    execs[v] = x[pos];
    uint32_t w = (uint32_t)(std::upper_bound(wb.begin(), wb.end(), pos) - wb.begin()) - 1;
    owner[v] = w;
    entry[v] = pos - wb[w];
  }
  if (wprog) {
    if (nworkers != L.nworkers) return fail(TG_EINVAL, "nworkers must be %u", L.nworkers);
    HIPCHK(hipMemcpy(wprog, L.wprog.p, (size_t)L.nworkers * 4, hipMemcpyDeviceToHost));
  }
  return TG_OK;
}

tg_status tg_emulate_schedule(const tg_graph* graphs, uint32_t ngraphs, uint32_t nworkers, uint32_t window,
                              uint32_t schedule, uint64_t seed, uint64_t* order, uint64_t* executed, uint64_t* makespan,
                              uint64_t* bound) {
  if (!graphs || !ngraphs || !order || !executed) return fail(TG_EINVAL, "NULL argument");
  if (window < 1 || window > 64 || nworkers == 0) return fail(TG_EINVAL, "window in [1,64], nworkers >= 1");
  std::vector<tg_graph> gs(graphs, graphs + ngraphs);
  for (auto g : gs) {
    if (!g) return fail(TG_EINVAL, "NULL graph");
    if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  }
  HostLayout H;
  tg_status s = plan_layout(gs, nworkers, schedule ? schedule : (uint32_t)TG_SCHED_LEVEL, H);
  if (s != TG_OK) return s;
  std::vector<uint32_t> ord(H.N);
  {
    HostLayout E = H;  // as the list executor runs it
    elide_list_edges(E);
    s = emulate_layout(E, window, seed, ord.data(), executed);
  }
  // report (graph, id), not positions
  std::vector<uint64_t> key_of(H.N);
  for (uint32_t gi = 0; gi < gs.size(); ++gi)
    for (uint32_t v = 0; v < gs[gi]->N(); ++v) key_of[H.pos_of[gi][v]] = ((uint64_t)gi << 32) | v;
  for (uint64_t i = 0; i < *executed; ++i) order[i] = key_of[ord[i]];
  if (s == TG_OK && makespan && bound) timed_makespan(gs, H, window, makespan, bound);
  return s;
}

tg_status tg_emulate_gang(const tg_graph* graphs, uint32_t ngraphs, uint32_t ngangs, uint32_t gang, uint32_t window,
                          uint32_t schedule, uint64_t seed, uint32_t elide, uint64_t* executed) {
  if (!graphs || !ngraphs || !executed) return fail(TG_EINVAL, "NULL argument");
  if (window < 1 || window > 64 || ngangs == 0 || gang < 1 || gang > tg::kMaxGang)
    return fail(TG_EINVAL, "window in [1,64], ngangs >= 1, gang in [1,%u]", tg::kMaxGang);
  std::vector<tg_graph> gs(graphs, graphs + ngraphs);
  for (auto g : gs) {
    if (!g) return fail(TG_EINVAL, "NULL graph");
    if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  }
  HostLayout H;
  tg_status s = plan_layout(gs, ngangs, schedule ? schedule : (uint32_t)TG_SCHED_LEVEL, H);
  if (s != TG_OK) return s;
  return emulate_gang_layout(H, gang, window, seed, elide != 0, executed);
}

tg_status tg_emulate_queue(const tg_graph* graphs, uint32_t ngraphs, uint32_t nworkers, uint32_t shards, uint32_t tile,
                           uint64_t seed, uint64_t* order, uint64_t* executed) {
  if (!graphs || !ngraphs || !order || !executed) return fail(TG_EINVAL, "NULL argument");
  if (nworkers == 0 || tile < 1 || tile > 64 || (shards != 1 && shards != 2 && shards != 4 && shards != 8))
    return fail(TG_EINVAL, "nworkers >= 1, tile in [1,64], shards 1, 2, 4 or 8");
  std::vector<tg_graph> gs(graphs, graphs + ngraphs);
  for (auto g : gs) {
    if (!g) return fail(TG_EINVAL, "NULL graph");
    if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  }
  HostLayout H;
  tg_status s = plan_layout(gs, 1, TG_SCHED_LEVEL, H);
  if (s != TG_OK) return s;
  std::vector<uint32_t> ord(H.N);
  s = emulate_queue(H, nworkers, shards, tile, seed, ord.data(), executed);
  std::vector<uint64_t> key_of(H.N);
  for (uint32_t gi = 0; gi < gs.size(); ++gi)
    for (uint32_t v = 0; v < gs[gi]->N(); ++v) key_of[H.pos_of[gi][v]] = ((uint64_t)gi << 32) | v;
  for (uint64_t i = 0; i < *executed; ++i) order[i] = key_of[ord[i]];
  return s;
}

tg_status tg_graph_exec_info(tg_graph g, uint32_t* workers, uint32_t* started) {
  if (!g || !workers || !started) return fail(TG_EINVAL, "NULL argument");
  if (!g->solo) return fail(TG_ESTATE, "graph was never executed");
  *workers = g->solo->nworkers;
  *started = g->solo->last_started;
  return TG_OK;
}

tg_status tg_graph_execute_comparator(tg_graph g, uint32_t mode, void* stream) {
  if (!g) return fail(TG_EINVAL, "graph is NULL");
  if (!g->finalized) return fail(TG_ESTATE, "graph not finalised");
  if (g->inflight) return fail(TG_EBUSY, "previous execution not waited for");
  if (mode != TG_CMP_PER_TASK && mode != TG_CMP_HIPGRAPH && mode != TG_CMP_HIPGRAPH_CAPTURED)
    return fail(TG_EINVAL, "unknown comparator %u", mode);
  tg_status s;
  if (!g->solo) {
    std::vector<tg_graph> gs{g};
    if ((s = build_layout(gs, Config(), g->solo)) != TG_OK) return s;
  }
  Layout& L = *g->solo;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t N = g->N();
  ExecParams P = L.params;
  if ((s = ensure_events(g)) != TG_OK) return s;
  HIPCHK(hipEventRecord(g->ev0, st));
  if (g->mode == TG_IMPLICIT) {
    HIPCHK(tg_launch_init_data(g->data.as<uint32_t>(), g->space, sm64_host(g->seed ^ (2ull << 32)), st));
  }
  // creation order is topological for the data edges; with anti-dependence
  // edges the level order the slots were assigned in is used
  auto task_at = [&](uint32_t i) { return g->anti ? g->topo[i] : i; };
  if (mode == TG_CMP_PER_TASK) {
    for (uint32_t i = 0; i < N; ++i) HIPCHK(tg::launch_one_task(P, L.pos_of[0][task_at(i)], st));
  } else if (mode == TG_CMP_HIPGRAPH_CAPTURED) {
    if (!g->hgcx) {
      // the per-task launch sequence, captured once from a private stream
      hipStream_t cs = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      for (uint32_t i = 0; i < N && ce == hipSuccess; ++i) ce = tg::launch_one_task(P, L.pos_of[0][task_at(i)], cs);
      hipGraph_t cg = nullptr;
      const hipError_t ee = hipStreamEndCapture(cs, &cg);
      (void)hipStreamDestroy(cs);
      if (ce != hipSuccess || ee != hipSuccess) {
        if (cg) (void)hipGraphDestroy(cg);
        return fail(TG_EDEVICE, "stream capture of the per-task launches: %s",
                    hipGetErrorString(ce != hipSuccess ? ce : ee));
      }
      g->hgc = cg;
      HIPCHK(hipGraphInstantiate(&g->hgcx, g->hgc, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(g->hgcx, st));
  } else {
    if (!g->hgx) {
      HIPCHK(hipGraphCreate(&g->hg, 0));
      std::vector<hipGraphNode_t> node(N);
      std::vector<hipGraphNode_t> deps;
      // predecessors over the executed edges
      std::vector<uint64_t> xp(N + 1, 0);
      for (uint32_t x : g->succ) xp[x + 1]++;
      for (uint32_t k = 0; k < N; ++k) xp[k + 1] += xp[k];
      std::vector<uint32_t> xpr(g->succ.size());
      {
        std::vector<uint64_t> fill(xp.begin(), xp.end() - 1);
        for (uint32_t j = 0; j < N; ++j)
          for (uint64_t a = g->succ_ptr[j]; a < g->succ_ptr[j + 1]; ++a) xpr[fill[g->succ[a]]++] = j;
      }
      for (uint32_t i = 0; i < N; ++i) {
        const uint32_t v = task_at(i);
        uint32_t pos = L.pos_of[0][v];
        void* args[2] = {(void*)&P, (void*)&pos};
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof(kp));
        kp.func = (void*)tg::one_task_kernel();
        kp.gridDim = dim3(1);
        kp.blockDim = dim3(64);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        deps.clear();
        for (uint64_t j = xp[v]; j < xp[v + 1]; ++j) deps.push_back(node[xpr[j]]);
        HIPCHK(hipGraphAddKernelNode(&node[v], g->hg, deps.empty() ? nullptr : deps.data(), deps.size(), &kp));
      }
      HIPCHK(hipGraphInstantiate(&g->hgx, g->hg, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(g->hgx, st));
  }
  HIPCHK(hipEventRecord(g->ev1, st));
  g->inflight = true;
  g->last_layout = nullptr;
  return TG_OK;
}

}  // extern "C"

// ================================================================ serving

// Continuous batching: a server thread admits submitted (compiled) graphs in
// arrival order while their device memory fits the budget, lays out each
// admitted group as one persistent launch on one of several streams, and
// retires launches as their completion events fire -- so requests that
// arrive while others run are admitted as soon as a launch slot and memory
// free up, and launches on different streams overlap on the device.  On
// completion a request's digests are copied to the host and its device
// memory is released.
struct tg_server_s {
  struct Req {
    tg_graph g = nullptr;
    uint64_t ticket = 0, bytes = 0;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    tg_status status = TG_OK;
    bool done = false;
    // the record lives until both its slot let go of it (a request can
    // finish while its launch still runs) and its waiter read it
    bool in_slot = false, waited = false;
  };
  // A launch slot: one stream, one layout at a time, and a builder thread
  // that compiles and launches the batch assigned to it, so that up to one
  // batch per slot is planned on the host at once.
  struct Slot {
    enum State { kIdle, kBuilding, kRunning };
    std::unique_ptr<Layout> lay;
    std::vector<Req*> reqs;
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr, ev0 = nullptr;  // end of the launch; its start (timing)
    State state = kIdle;
    bool assigned = false;  // a batch waits for the builder
    bool reports = false;   // the launch reports graphs as they finish (flags in the layout)
    // device memory of requests completed while their launch still runs,
    // freed when it ends
    std::vector<std::unique_ptr<DevBuf>> keep;
    std::condition_variable cv;
    std::thread th;
  };
  static constexpr uint32_t kLargeTasks = 1u << 16;  // size class served by slot 0 alone
  uint64_t budget = 0, in_use = 0, next_ticket = 1;
  uint32_t workers = 0, max_batch = 64;
  // launch configuration of every batch: the ready queue with records built
  // on the device (no host schedule), unless lists are chosen
  Config cfg;
  std::vector<std::unique_ptr<Slot>> slots;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::unordered_set<tg_graph> live;  // graphs of requests not yet finished
  std::mutex mu;
  std::condition_variable cv_done, cv_work;
  std::thread th;
  bool stop = false;
  uint64_t tasks_done = 0, launches = 0, peak_in_use = 0;
  // host time of the serving thread by phase, and executor time on the device
  double build_ms = 0, launch_ms = 0, retire_ms = 0, gpu_ms = 0;
  // parts of it: schedules and records, allocator hooks, host-device copies;
  // device-built layouts: the graphs' buffers, the layout's tables and kernels
  double plan_ms = 0, hook_ms = 0, copy_ms = 0, setup_ms = 0, tables_ms = 0;
};

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Device bytes a compiled graph occupies while admitted: its payloads (or
// array) and digests plus its share of a layout.
uint64_t graph_device_bytes(tg_graph g) {
  const uint64_t N = g->N(), E = g->succ.size(), P = g->dpred.size();
  uint64_t b = N * 4;  // digests
  b += g->mode == TG_EXPLICIT ? (uint64_t)g->nslots * g->n * 4ull : g->space * 4ull;
  b += g->blob.size() * 4;  // the compiled graph on the device
  // its share of a launch: records, counters and reset values, successor
  // positions, predecessor addresses, a slot in each of 8 queue shards
  b += N * (sizeof(TaskRec) + 4 + 4 + 8 * 4) + E * 4 + P * 8;
  return b + 4096;
}

// Copies a served graph's digests to the host and releases its device
// memory -- or, with `keep`, hands the memory to the caller (a launch that
// still runs may hold addresses inside it), leaving the graph free to be
// submitted again.
void release_graph_device(tg_graph g, std::vector<std::unique_ptr<DevBuf>>* keep = nullptr) {
  const uint32_t N = g->N();
  g->host_digest.assign(N, 0);
  if (N && g->digest.p) (void)hipMemcpy(g->host_digest.data(), g->digest.p, (size_t)N * 4, hipMemcpyDeviceToHost);
  for (DevBuf* b : {&g->payload, &g->data, &g->digest, &g->dblob}) {
    if (keep && b->p) {
      keep->push_back(std::make_unique<DevBuf>());
      keep->back()->take(*b);
    }
    b->release();
  }
  drop_solo(g);
  g->inflight = false;
  g->released = true;
}

// Marks a request finished (the server's lock is held): its graph may be
// submitted again.
void finish_req(tg_server srv, tg_server_s::Req* r, tg_status st, uint64_t t) {
  r->status = st;
  r->t_done = t;
  r->done = true;
  srv->live.erase(r->g);
}

// A slot lets go of a request record (the server's lock is held): freed now
// if its waiter has already read it, else by the waiter.
void leave_slot(tg_server srv, tg_server_s::Req* r) {
  r->in_slot = false;
  if (r->waited) srv->reqs.erase(r->ticket);
}

// Builder thread of one slot: compile the assigned batch into a layout and
// launch it on the slot's stream.
void slot_builder(tg_server srv, tg_server_s::Slot* sl) {
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    sl->cv.wait(lk, [&] { return sl->assigned || srv->stop; });
    if (!sl->assigned) return;  // stopping
    sl->assigned = false;
    const std::vector<tg_server_s::Req*> batch = sl->reqs;
    const Config cfg = srv->cfg;
    lk.unlock();
    std::vector<tg_graph> gs;
    for (auto* r : batch) gs.push_back(r->g);
    const bool device_built = cfg.dispatch == TG_DISPATCH_QUEUE;
    const uint64_t h0 = t_hook_ns, c0 = t_copy_ns, s0 = t_setup_ns, b0 = t_tables_ns;
    const uint64_t t0 = now_ns();
    t_copy_stream = sl->st;
    tg_status st;
    sl->reports = device_built;
    if (device_built) {
      if (!sl->lay) sl->lay = std::make_unique<Layout>();
      st = build_layout_device(gs, cfg, *sl->lay, sl->st, true);
    } else {
      st = build_layout(gs, cfg, sl->lay, nullptr, false);
    }
    t_copy_stream = nullptr;
    const uint64_t t1 = now_ns();
    if (st == TG_OK && hipEventRecord(sl->ev0, sl->st) != hipSuccess) st = TG_EDEVICE;
    if (st == TG_OK) st = launch_layout(*sl->lay, cfg, gs, sl->st);
    if (st == TG_OK && hipEventRecord(sl->ev, sl->st) != hipSuccess) st = TG_EDEVICE;
    const uint64_t t2 = now_ns();
    if (st != TG_OK)
      for (auto* r : batch) release_graph_device(r->g);
    lk.lock();
    srv->build_ms += (t1 - t0) * 1e-6;
    srv->launch_ms += (t2 - t1) * 1e-6;
    if (sl->lay) srv->plan_ms += sl->lay->plan_ms;
    srv->hook_ms += (t_hook_ns - h0) * 1e-6;
    srv->copy_ms += (t_copy_ns - c0) * 1e-6;
    srv->setup_ms += (t_setup_ns - s0) * 1e-6;
    srv->tables_ms += (t_tables_ns - b0) * 1e-6;
    if (st != TG_OK) {
      for (auto* r : batch) {
        srv->in_use -= r->bytes;
        finish_req(srv, r, st, now_ns());
        leave_slot(srv, r);
      }
      sl->lay.reset();
      sl->reqs.clear();
      sl->state = tg_server_s::Slot::kIdle;
      srv->cv_done.notify_all();
    } else {
      sl->state = tg_server_s::Slot::kRunning;
      srv->launches++;
    }
    srv->cv_work.notify_all();
  }
}

// Serving thread: retires finished launches and admits waiting requests,
// by memory budget, into idle slots (their builders do the rest).
void server_loop(tg_server srv) {
  std::unique_lock<std::mutex> lk(srv->mu);
  while (!srv->stop) {
    bool progressed = false, running = false;
    // requests whose graphs finished inside launches that still run
    for (auto& slp : srv->slots) {
      tg_server_s::Slot& sl = *slp;
      if (sl.state != tg_server_s::Slot::kRunning || !sl.reports || !sl.lay || !sl.lay->gflag) continue;
      const uint32_t seq = sl.lay->gseq;
      for (size_t i = 0; i < sl.reqs.size() && i < sl.lay->gflag_n; ++i) {
        tg_server_s::Req* r = sl.reqs[i];
        if (r->done || __atomic_load_n(sl.lay->gflag + i, __ATOMIC_ACQUIRE) != seq) continue;
        const uint64_t t = now_ns();
        lk.unlock();
        release_graph_device(r->g, &sl.keep);
        lk.lock();
        srv->tasks_done += r->g->N();
        finish_req(srv, r, TG_OK, t);
        progressed = true;
        srv->cv_done.notify_all();
      }
    }
    // retire finished launches
    for (auto& slp : srv->slots) {
      tg_server_s::Slot& sl = *slp;
      if (sl.state != tg_server_s::Slot::kRunning) continue;
      running = true;
      if (hipEventQuery(sl.ev) != hipSuccess) continue;
      const uint64_t t = now_ns(), h0 = t_hook_ns, c0 = t_copy_ns;
      float gms = 0;
      if (hipEventElapsedTime(&gms, sl.ev0, sl.ev) == hipSuccess) srv->gpu_ms += gms;
      tg_status st = check_abort(sl.lay.get());
      std::vector<tg_server_s::Req*> done;
      done.swap(sl.reqs);
      lk.unlock();
      for (auto* r : done)
        if (!r->done) release_graph_device(r->g);
      sl.keep.clear();
      // a device-built layout keeps its buffers for the slot's next batch
      if (sl.lay && sl.lay->cfg.dispatch != TG_DISPATCH_QUEUE) sl.lay.reset();
      lk.lock();
      for (auto* r : done) {
        srv->in_use -= r->bytes;
        if (!r->done) {  // else reported while the launch ran
          srv->tasks_done += r->g->N();
          finish_req(srv, r, st, t);
        }
        leave_slot(srv, r);
      }
      sl.state = tg_server_s::Slot::kIdle;
      srv->retire_ms += (now_ns() - t) * 1e-6;
      srv->hook_ms += (t_hook_ns - h0) * 1e-6;
      srv->copy_ms += (t_copy_ns - c0) * 1e-6;
      progressed = true;
      srv->cv_done.notify_all();
    }
    // requests that can never fit the budget fail at once
    for (auto it = srv->pending.begin(); it != srv->pending.end();) {
      if ((*it)->bytes > srv->budget) {
        finish_req(srv, *it, TG_ENOMEM, now_ns());
        srv->cv_done.notify_all();
        it = srv->pending.erase(it);
      } else {
        ++it;
      }
    }
    // admit waiting requests into idle slots, in arrival order and while
    // the budget holds them.  With several slots, requests of at least
    // kLargeTasks tasks go to slot 0 only (which takes small ones when no
    // large one waits): a small request then never shares a launch -- and
    // its ready queue -- with a graph that keeps the launch busy for long.
    for (size_t si = 0; si < srv->slots.size(); ++si) {
      tg_server_s::Slot& sl = *srv->slots[si];
      if (sl.state != tg_server_s::Slot::kIdle || srv->pending.empty()) continue;
      const bool sized = srv->slots.size() > 1;
      auto large = [](const tg_server_s::Req* r) { return r->g->N() >= tg_server_s::kLargeTasks; };
      bool want_large = false;
      if (sized && si == 0)
        for (auto* r : srv->pending) want_large |= large(r);
      std::vector<tg_server_s::Req*> batch;
      uint64_t add = 0;
      for (auto it = srv->pending.begin(); it != srv->pending.end() && batch.size() < srv->max_batch;) {
        tg_server_s::Req* r = *it;
        if (sized && large(r) != want_large) {
          ++it;
          continue;
        }
        if (srv->in_use + add + r->bytes > srv->budget) break;
        batch.push_back(r);
        add += r->bytes;
        it = srv->pending.erase(it);
      }
      if (batch.empty()) continue;
      srv->in_use += add;
      if (srv->in_use > srv->peak_in_use) srv->peak_in_use = srv->in_use;
      const uint64_t t = now_ns();
      for (auto* r : batch) {
        r->t_admit = t;
        r->in_slot = true;
      }
      sl.reqs = batch;
      sl.state = tg_server_s::Slot::kBuilding;
      sl.assigned = true;
      sl.cv.notify_one();
      progressed = true;
    }
    if (progressed) continue;
    if (running) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      srv->cv_work.wait(lk);  // woken by submissions, builders and destroy
    }
  }
}

}  // namespace

extern "C" {

tg_status tg_server_create(tg_server* out, uint64_t budget_bytes, uint32_t slots, uint32_t max_batch) {
  if (!out) return fail(TG_EINVAL, "out is NULL");
  *out = nullptr;
  if (slots == 0) slots = 4;
  if (slots > 4) return fail(TG_EINVAL, "at most 4 launch slots (one hardware queue each)");
  if (budget_bytes == 0) return fail(TG_EINVAL, "budget must be positive");
  uint32_t resident = 0;
  tg_status s = resident_workers(TG_MAP_WAVE, 4, &resident);
  if (s != TG_OK) return s;
  auto srv = std::make_unique<tg_server_s>();
  srv->budget = budget_bytes;
  srv->workers = resident / slots;  // concurrent launches stay co-resident together
  srv->cfg.workers = srv->workers;
  srv->cfg.dispatch = TG_DISPATCH_QUEUE;
  srv->max_batch = max_batch ? max_batch : 64;
  for (uint32_t i = 0; i < slots; ++i) {
    auto sl = std::make_unique<tg_server_s::Slot>();
    HIPCHK(hipStreamCreateWithFlags(&sl->st, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&sl->ev));
    HIPCHK(hipEventCreate(&sl->ev0));
    srv->slots.push_back(std::move(sl));
  }
  tg_server srvp = srv.release();
  for (auto& sl : srvp->slots) sl->th = std::thread(slot_builder, srvp, sl.get());
  srvp->th = std::thread(server_loop, srvp);
  *out = srvp;
  return TG_OK;
}

tg_status tg_server_configure(tg_server srv, const tg_exec_config* cfgp) {
  if (!srv || !cfgp) return fail(TG_EINVAL, "NULL argument");
  Config c = resolve(cfgp);
  if (!cfgp->dispatch) c.dispatch = TG_DISPATCH_QUEUE;
  if (!cfgp->workers) c.workers = srv->workers;
  tg_status s = check_config(c);
  if (s != TG_OK) return s;
  if (c.mapping == TG_MAP_GANG) return fail(TG_EINVAL, "the server runs wavefront or workgroup workers");
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->cfg = c;
  return TG_OK;
}

tg_status tg_server_submit(tg_server srv, tg_graph g, uint64_t* ticket) {
  if (!srv || !g || !ticket) return fail(TG_EINVAL, "NULL argument");
  if (!g->finalized) return fail(TG_ESTATE, "submit compiled graphs (tg_graph_finalize first)");
  if (g->inflight) return fail(TG_EBUSY, "graph has an execution in flight");
  auto r = std::make_unique<tg_server_s::Req>();
  r->g = g;
  r->bytes = graph_device_bytes(g);
  r->t_submit = now_ns();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (!srv->live.insert(g).second) return fail(TG_EBUSY, "graph already submitted and not finished");
  r->ticket = srv->next_ticket++;
  *ticket = r->ticket;
  srv->pending.push_back(r.get());
  srv->reqs[r->ticket] = std::move(r);
  srv->cv_work.notify_one();
  return TG_OK;
}

tg_status tg_server_wait(tg_server srv, uint64_t ticket, uint64_t* submit_ns, uint64_t* admit_ns, uint64_t* done_ns) {
  if (!srv) return fail(TG_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return fail(TG_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  tg_server_s::Req* r = it->second.get();
  srv->cv_done.wait(lk, [&] { return r->done; });
  if (submit_ns) *submit_ns = r->t_submit;
  if (admit_ns) *admit_ns = r->t_admit;
  if (done_ns) *done_ns = r->t_done;
  const tg_status st = r->status;
  if (r->in_slot) r->waited = true;  // the slot's retirement frees it
  else srv->reqs.erase(it);
  if (st != TG_OK) return fail(st, "request %llu failed", (unsigned long long)ticket);
  return TG_OK;
}

tg_status tg_server_stats(tg_server srv, uint64_t* tasks_done, uint64_t* launches, uint64_t* peak_bytes,
                          double* phase_ms) {
  if (!srv) return fail(TG_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (tasks_done) *tasks_done = srv->tasks_done;
  if (launches) *launches = srv->launches;
  if (peak_bytes) *peak_bytes = srv->peak_in_use;
  if (phase_ms) {
    phase_ms[0] = srv->build_ms;
    phase_ms[1] = srv->launch_ms;
    phase_ms[2] = srv->retire_ms;
    phase_ms[3] = srv->gpu_ms;
    phase_ms[4] = srv->plan_ms;
    phase_ms[5] = srv->hook_ms;
    phase_ms[6] = srv->copy_ms;
    phase_ms[7] = srv->setup_ms;
    phase_ms[8] = srv->tables_ms;
  }
  return TG_OK;
}

tg_status tg_server_destroy(tg_server srv) {
  if (!srv) return TG_OK;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    // let admitted and pending work finish
    srv->cv_done.wait(lk, [&] {
      if (!srv->pending.empty()) return false;
      for (auto& sl : srv->slots)
        if (sl->state != tg_server_s::Slot::kIdle) return false;
      return true;
    });
    srv->stop = true;
    srv->cv_work.notify_all();
    for (auto& sl : srv->slots) sl->cv.notify_all();
  }
  srv->th.join();
  for (auto& sl : srv->slots) {
    sl->th.join();
    if (sl->ev) (void)hipEventDestroy(sl->ev);
    if (sl->ev0) (void)hipEventDestroy(sl->ev0);
    if (sl->st) (void)hipStreamDestroy(sl->st);
  }
  delete srv;
  return TG_OK;
}

}  // extern "C"
