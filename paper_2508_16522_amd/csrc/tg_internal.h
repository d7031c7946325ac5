// Internal layout shared by the host compiler (tg_host.cpp) and the kernels.
//
// A "layout" is a compiled schedule (Algorithm 1, Compile) of one or more
// graphs for one launch configuration.  Every task of every graph gets a
// position; positions are grouped per worker (a wavefront or a workgroup, the
// GPU counterpart of the paper's per-resource worker actor), and within a
// worker they are in the order the schedule runs them (topological).  Each position owns one u32
// counter of pending in-edges (Algorithm 1's per-vertex counter) and an O(1)
// out-edge list of successor positions.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tg {

// Per-graph constants.
struct GraphEnt {
  uint64_t key1;     // sm64(seed ^ (1 << 32)): explicit initial payload key
  uint64_t key2;     // sm64(seed ^ (2 << 32)): implicit initial array key
  uint32_t* digest;  // digest[task id]
  uint32_t* data;    // implicit: shared array A (index space words)
  uint32_t n;        // explicit: payload words per task (power of two)
  uint32_t mode;     // 1 explicit, 2 implicit
  uint32_t nsinks;   // tasks without out-edges (per-graph completion)
  uint32_t pad;
};

constexpr uint32_t kInPred = 6;  // predecessor payload addresses held in the record
constexpr uint32_t kInSucc = 8;  // successor positions held in the record

// Per-position task record: 128 bytes (32 dwords), read by one coalesced
// vector load per wavefront (lane i holds dword i % 32) and unpacked with
// readlane.  The first kInPred predecessor addresses and kInSucc successor
// positions are inline, so a task's payload loads depend on one load (the
// record) and its edge signals on none after the payload store.
struct alignas(128) TaskRec {
  uint64_t out;            // dw 0-1  explicit: device address of this task's payload
                           //         implicit: device address of its first region requirement
  uint32_t tid;            // dw 2    task id inside its graph (creation index)
  uint32_t graph;          // dw 3    index into the graph table
  uint32_t pred_beg;       // dw 4    explicit: all predecessors at pred_addr[pred_beg ..]
  uint32_t npred;          // dw 5    number of distinct predecessors (= in-degree)
  uint32_t succ_beg;       // dw 6    all successors at succ_pos[succ_beg ..]
  uint32_t nsucc;          // dw 7    number of successors
  uint32_t rounds;         // dw 8    mix rounds
  uint32_t nreq;           // dw 9    implicit: number of region requirements
  uint64_t pred[kInPred];  // dw 10-21 first predecessors' payload addresses
  uint32_t succ[kInSucc];  // dw 22-29 first successor positions
  uint32_t pad[2];         // dw 30-31
};
static_assert(sizeof(TaskRec) == 128, "task record is 32 dwords");
enum : uint32_t {
  kDwOut = 0, kDwTid = 2, kDwGraph = 3, kDwPredBeg = 4, kDwNpred = 5, kDwSuccBeg = 6, kDwNsucc = 7,
  kDwRounds = 8, kDwNreq = 9, kDwPred = 10, kDwSucc = 22
};
static_assert(offsetof(TaskRec, tid) == 4 * kDwTid && offsetof(TaskRec, graph) == 4 * kDwGraph &&
                  offsetof(TaskRec, pred_beg) == 4 * kDwPredBeg && offsetof(TaskRec, npred) == 4 * kDwNpred &&
                  offsetof(TaskRec, succ_beg) == 4 * kDwSuccBeg && offsetof(TaskRec, nsucc) == 4 * kDwNsucc &&
                  offsetof(TaskRec, rounds) == 4 * kDwRounds && offsetof(TaskRec, nreq) == 4 * kDwNreq &&
                  offsetof(TaskRec, pred) == 4 * kDwPred && offsetof(TaskRec, succ) == 4 * kDwSucc,
              "record dword map");

// Region requirement on the device (implicit mode).
struct alignas(16) ReqDev {
  uint64_t lo, hi;  // [lo, hi)
  uint32_t priv;    // 1 RO, 2 RW
  uint32_t rw_base; // ordinal of this interval's first element among the
                    // task's written elements (digest weights)
  uint32_t pad[2];
};

// Control block written by the kernels.
struct Ctrl {
  uint32_t abort;      // set when a worker's watchdog fired
  uint32_t started;    // workers that began (diagnostic launches only)
  uint32_t stuck_worker, stuck_pos, stuck_cnt, stuck_h, stuck_wcnt;  // first abort
  uint32_t resident;   // residency probe: workers that saw every worker check in
  uint32_t sticky;     // aborts of earlier launches since the host last looked
  uint32_t precond;    // 1 + index of the pre-condition flag not met in time (0: none)
  uint32_t pad0[22];
  // device clock (s_memrealtime) of the most recent task start any worker
  // published (atomic max; each worker publishes at most once per
  // ExecParams::progress_ticks); on its own 128-byte line
  uint64_t progress;
  uint32_t pad1[30];
};
static_assert(sizeof(Ctrl) == 256 && offsetof(Ctrl, progress) == 128, "control block layout");

struct ExecParams {
  const TaskRec* rec;
  const uint64_t* pred_addr;   // payload addresses of predecessors
  const uint32_t* succ_pos;    // successor positions
  const uint32_t* indeg;       // initial counter values
  uint32_t* cnt;               // pending in-edge counters
  const uint32_t* wbase;       // worker w owns positions [wbase[w], wbase[w+1])
  const GraphEnt* gtab;
  Ctrl* ctrl;
  const uint32_t* owner;       // worker of every position
  uint32_t* bell;              // per-worker doorbell, one per 128-byte line
  uint32_t npos;
  uint32_t nworkers;
  uint32_t window;             // 1..64
  uint32_t spin_limit;         // 0 = no limit
  uint32_t diag;               // 1: count started workers
  uint32_t idle_sleep;         // s_sleep(2) steps between empty polls after 64 of them
  uint32_t notify;             // 1: zeroing decrements ring the owner's doorbell
  uint32_t residency_probe;    // 1: check in, wait for all workers (bounded), exit
  uint32_t gang;               // workgroups per gang (mapping 3), else 1; with gangs the
                               // counters start at in-degree x gang and digests are
                               // sums of the members' parts
  uint64_t watchdog_ticks;     // s_memrealtime ticks (100 MHz)
  uint64_t progress_ticks;     // a worker publishes Ctrl::progress at most this often
  // ready-queue dispatch (kernels k_exec_wave_q / k_exec_block_q)
  uint32_t* q;                 // qshards x qcap ticket slots (kQEmpty when free)
  uint32_t* qctl;              // shard s: head at qctl[s * kQLine], tail at
                               // qctl[(qshards + s) * kQLine]; sinks finished
                               // at qctl[2 * qshards * kQLine]
  const uint32_t* qsrc;        // positions without in-edges (pushed at reset)
  uint32_t nsrc;
  uint32_t nsinks;             // positions without out-edges
  uint32_t qshards;            // power of two, 1..8
  uint32_t qcap;               // slots per shard: the task count plus the exit sentinels
  uint32_t qtile;              // tickets claimed per pop (1..64)
  uint32_t qsent;              // exit sentinels pushed into every shard at the end
  // per-graph completion (queue kernels; null gdone: not reported)
  uint32_t* gdone;             // sinks finished per graph of the layout
  uint32_t* gflag;             // per graph, in host memory: gseq once it finished
  uint32_t gseq;
  uint32_t gated;              // 1: a pre-condition wait precedes the launch; workers
                               // leave at once if it gave up (Ctrl::abort set)
  // diagnostics, last: the kernels read them rarely, and with these four
  // pointers after the fields the executors read on every task the compiler
  // keeps more of the latter in scalar registers (fewer spills)
  uint32_t* execs;             // diagnostics: executions per position (or null)
  uint32_t* wprog;             // diagnostics: list entries finished per worker (or null)
  uint64_t* tstamp;            // diagnostics: per position [start, end] realtime (or null)
  uint64_t* wstamp;            // diagnostics: per worker [first poll, last scan, scans, bell reads]
};

// Pre-condition flags of one launch (words in pinned host memory mapped for
// the device): the launch may start once every *addr[i] >= value[i].
constexpr uint32_t kMaxPreFlags = 8;
struct FlagWait {
  const uint32_t* addr[kMaxPreFlags];
  uint32_t value[kMaxPreFlags];
  uint32_t n;
};

// One graph of a layout whose task records are built on the device
// (k_build_records) from the graph's compiled blob: row offsets and id lists
// of its distinct predecessors (explicit) and executed successors, counter
// reset values, mix rounds, payload slots (or null), requirement rows and
// requirements (implicit), and sources.
struct alignas(16) GraphSrc {
  const uint32_t* pred_ptr;
  const uint32_t* preds;
  const uint32_t* succ_ptr;
  const uint32_t* succ;
  const uint32_t* indeg;
  const uint32_t* rounds;
  const uint32_t* slot;
  const uint32_t* req_ptr;
  const ReqDev* reqs;
  const uint32_t* src;
  uint64_t payload;     // explicit: payload base address; slot or task v at payload + 4n v
  uint32_t pos_base;    // first position of the graph in the layout
  uint32_t pred_base;   // first entry of its predecessor addresses in pred_addr
  uint32_t succ_base;   // first entry of its successor positions in succ_pos
  uint32_t src_base;    // first entry of its sources in the launch's source list
  uint32_t n;           // payload words (explicit)
  uint32_t mode;
  uint32_t pad[2];
};

// List dispatch: counter bit meaning "this list entry also waits for the
// entry before it in its worker's list".  That predecessor runs on the same
// worker, which finishes it before taking this task, so its edge is not
// counted (the layout drops it from the predecessor's successors); the bits
// below hold the other in-edges still pending.
constexpr uint32_t kAfterPrev = 0x80000000u;
constexpr uint32_t kPendingMask = 0x7FFFFFFFu;

constexpr uint32_t kQEmpty = 0xFFFFFFFFu;
constexpr uint32_t kQExit = 0xFFFFFFFEu;  // exit sentinel
constexpr uint32_t kQLine = 32;           // u32 words between queue control words (128 bytes)

constexpr uint32_t kBellStride = 32;  // u32 words between doorbells (128 bytes)
constexpr uint32_t kMaxGang = 32;  // workgroups per gang (mapping 3)

// Launchers (tg_kernels.hip).  All return hipError_t of the launch.
// mapping 1: one wavefront per task; 2: one workgroup of wg_waves wavefronts;
// 3: a gang of p.gang such workgroups (grid_blocks = workers x gang).
hipError_t launch_reset(const ExecParams& p, hipStream_t s);
// One wavefront waits until every pre-condition flag is met, for at most
// timeout_ticks (s_memrealtime, 100 MHz); on time-out it raises ctrl->abort
// and records the flag in ctrl->precond.
hipError_t launch_wait_flags(const FlagWait& fw, Ctrl* ctrl, uint64_t timeout_ticks, hipStream_t s);
// Stores value into *flag (system scope, after a system-scope release) unless
// ctrl->abort is set (the launch before it in stream order was abandoned).
hipError_t launch_set_flag(uint32_t* flag, uint32_t value, const Ctrl* ctrl, hipStream_t s);
hipError_t launch_exec(const ExecParams& p, uint32_t mapping, uint32_t wg_waves, uint32_t grid_blocks,
                       hipStream_t s);
// Ready-queue dispatch: clear the slots used by the previous launch, then
// seed the queue with the sources (after launch_reset, before the executor).
hipError_t launch_queue_reset(const ExecParams& p, hipStream_t s);
// Only the clearing half: empties the slots the last launch of p filled.
hipError_t launch_queue_clear(const ExecParams& p, hipStream_t s);
hipError_t launch_exec_queue(const ExecParams& p, uint32_t mapping, uint32_t wg_waves, uint32_t grid_blocks,
                             hipStream_t s);
// Task records, predecessor addresses, successor positions, counter reset
// values and the source list of a layout, built on the device from the
// graphs' blobs: ng graphs (table gsrc, ascending pos_base and src_base),
// npos positions, nsrc sources.
hipError_t launch_build_records(const GraphSrc* gsrc, uint32_t ng, uint32_t npos, uint32_t nsrc, TaskRec* rec,
                                uint64_t* pred_addr, uint32_t* succ_pos, uint32_t* indeg, uint32_t* src,
                                hipStream_t s);
// Clears n words to v with a kernel (stream-ordered, no memset node).
hipError_t launch_fill(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// Occupancy: blocks per CU for the executor kernel of this mapping.
int exec_blocks_per_cu(uint32_t mapping, uint32_t wg_waves);
// One task per launch (comparator): runs position `pos` with no counters.
hipError_t launch_one_task(const ExecParams& p, uint32_t pos, hipStream_t s);
const void* one_task_kernel();

}  // namespace tg

#include <string>
#include <vector>

#include "taskgraph.h"

// Records the message of a failure for tg_last_error() on the calling thread
// and returns s (tg_host.cpp).
tg_status tg_set_error(tg_status s, const char* fmt, ...);

// Result of device dependence inference: out-edge CSR, rows ascending.
struct InferResult {
  std::vector<uint64_t> row_ptr;
  std::vector<uint32_t> col;
  double ms = 0;  // device time of the inference kernels
};
// Dependence inference of a finalised implicit graph (tg_infer.hip):
// requirements req_ptr[N+1] / reqs[n_reqs] (tg_region_req records) in host
// memory, DAG returned in host memory, device buffers allocated per call.
tg_status tg_infer_dag_host(uint32_t N, const uint64_t* req_ptr, const void* reqs, uint64_t n_reqs, uint64_t space,
                            InferResult& res);
hipError_t tg_launch_init_data(uint32_t* A, uint64_t space, uint64_t key2, hipStream_t s);
