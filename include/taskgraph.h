/*
 * taskgraph.h -- C ABI of the MI355X (gfx950) task-DAG executor.
 *
 * The calls follow the paper's statement of the problem (Yadav et al., "On the
 * Duality of Task and Actor Programming Models"):
 *   - Figure 3 and Section 2: every operation returns an event for its
 *     completion and is predicated on a set of earlier events.  Here an event
 *     is the creation index of the task that produces it.
 *   - Section 4.1: a graph of operations is built dynamically, registered
 *     (finalised, i.e. compiled) once and then launched as one operation, as
 *     often as needed.
 *   - Algorithm 1: compilation gives every vertex an atomic counter of pending
 *     in-edges and an O(1) out-edge index; execution resets the counters,
 *     starts the vertices without in-edges, decrements one counter per edge
 *     and runs a vertex when its counter reaches zero.
 *   - Section 2 (implicitly parallel systems) and Section 5: instead of
 *     events, tasks may declare the data they read and write; the runtime
 *     infers the dependences, and the result equals sequential program order.
 *
 * Task body (the paper's Task Bench tasks run a floating-point busy loop,
 * Section 6.1; this library runs an exact integer body so every result is
 * reproducible bit for bit):
 *   mix_round(x) = xorshift32_{13,17,5}(x) * 0x9E3779B1 + 0x7F4A7C15 (mod 2^32)
 *   h32(s,t,i)   = low32(sm64(sm64(s ^ (t << 32)) ^ i)), sm64 = SplitMix64
 *   explicit task v with payload of n words:
 *     in[k]  = h32(seed, 1, (v << 16) | k)            if v has no predecessor
 *            = sum over distinct predecessors p of out_p[k]   (mod 2^32)
 *     out[k] = mix_round^R(in[k] ^ v)
 *     digest = sum_k out[k] * (2k + 1)                (mod 2^32)
 *   implicit task k on the shared array A (initially A[e] = h32(seed, 2, e)):
 *     c = sum of A[e] over its read-only elements;
 *     each read-write element e (declaration order): A[e] = mix^R(A[e]^c^k);
 *     digest = sum_j A_new[e_j] * (2j + 1), j enumerating written elements.
 *   checksum = sum_v digest(v) * (2v + 1)             (mod 2^64)
 *
 * Conventions.
 *   - Every call returns tg_status; 0 is success, negative values are errors.
 *     tg_status_str() names a status; tg_last_error() gives the message of the
 *     most recent failure on the calling thread.
 *   - Pointers named host_* / const arrays of the build calls are host memory
 *     owned by the caller and copied before the call returns.  Device memory
 *     is owned by the library (allocated through the allocator set with
 *     tg_set_allocator, else hipMalloc) and freed by the matching destroy.
 *   - Streams are hipStream_t passed as void*; NULL is the default stream.
 *   - A handle may be used by one thread at a time.
 *   - All kernels bound every wait: a wait that sees no progress for the
 *     configured watchdog interval aborts the launch, and the following
 *     wait/read call returns TG_ETIMEOUT.
 */
#ifndef TASKGRAPH_H
#define TASKGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tg_status;
enum {
  TG_OK = 0,
  TG_EINVAL = -1,    /* bad argument: unknown event, bad interval, wrong mode */
  TG_ENOMEM = -2,    /* device or host allocation failed, or budget exceeded */
  TG_EBUSY = -3,     /* graph already finalised / execution in flight */
  TG_EDEVICE = -4,   /* a HIP runtime call failed (message in tg_last_error) */
  TG_ETIMEOUT = -5,  /* the device watchdog aborted a launch */
  TG_ESTATE = -6     /* call not valid in the current state (e.g. not finalised) */
};

typedef struct tg_graph_s* tg_graph;
typedef struct tg_batch_s* tg_batch;
typedef struct tg_server_s* tg_server;
typedef struct tg_flag_s* tg_flag;
typedef uint32_t tg_event; /* creation index of the producing task in its graph */

enum { TG_EXPLICIT = 1, TG_IMPLICIT = 2 };
enum { TG_RO = 1, TG_RW = 2 };

/* Region requirement: half-open interval [lo, hi) of the graph's index space
 * with privilege TG_RO or TG_RW (Section 2, implicitly parallel systems). */
typedef struct {
  uint64_t lo, hi;
  uint32_t priv;
  uint32_t _pad;
} tg_region_req;

/* Launch configuration of the persistent executor.  Zero fields mean "let the
 * library choose" (built-in defaults).
 *   mapping      : 1 = one wavefront per task, 2 = one workgroup per task,
 *                  3 = a gang of `gang` workgroups (on different CUs) per task.
 *   workers      : number of workers (wavefronts, workgroups or gangs); 0 = as many
 *                  as are co-resident (calibrated, see tg_exec_occupancy);
 *                  larger values are clamped to that.
 *   window       : ready-window length scanned per poll (1..64).
 *   wg_waves     : wavefronts per workgroup for mappings 2 and 3 (1..16).
 *   watchdog_ms  : abort a launch after this long without progress.
 *   spin_limit   : if non-zero, abort after this many consecutive empty polls
 *                  (lets a host test force the timeout path).
 *   diag         : 1 = diagnostic launch (per-task execution counts and
 *                  timestamps, readable with tg_graph_debug_*).
 *   notify       : 1 = the decrement that empties a counter also rings the
 *                  owning worker's doorbell, and idle workers poll only their
 *                  doorbell (fewer polls, one more hop per task).
 *   idle_sleep   : back-off of an idle worker, in units of 128 cycles
 *                  (1..64, default 2), after its first 64 empty polls; with
 *                  the lists it doubles after every further 64 empty polls,
 *                  up to 32 times this value (at most 256 units).
 *   schedule     : how tasks are partitioned over the workers' lists
 *                  (Algorithm 1, Compile): TG_SCHED_LEVEL (default) sorts by
 *                  dependence level and deals round-robin; TG_SCHED_SPREAD
 *                  stretches every graph's levels over the same interval
 *                  before sorting and dealing, so graphs of different depths
 *                  advance side by side; TG_SCHED_LIST simulates the workers
 *                  with estimated task costs and starts ready tasks
 *                  longest-remaining-path first; TG_SCHED_COLUMN gives task i
 *                  of every level of a graph to the same worker (graphs packed
 *                  side by side by width) and orders each worker's list by the
 *                  stretched level, so columns stay on one worker and shallow
 *                  graphs fill the gaps of deep ones; TG_SCHED_BALANCED keeps
 *                  the level order but gives each task to the worker with the
 *                  least estimated work so far (tasks of very different
 *                  costs).
 *   gang         : mapping 3: workgroups per gang (2..32).  Every member runs
 *                  the scheduling loop of the gang's list, executes its share
 *                  of each task's work items and signals the task's out-edges
 *                  itself (a counter starts at in-degree x gang; TG_EINVAL if
 *                  that exceeds 2^31 - 1); the digest is the sum of the
 *                  members' parts. */
typedef struct {
  uint32_t mapping;
  uint32_t workers;
  uint32_t window;
  uint32_t wg_waves;
  uint32_t watchdog_ms;
  uint32_t spin_limit;
  uint32_t diag;
  uint32_t notify;
  uint32_t idle_sleep;
  uint32_t schedule;
  uint32_t gang;
  uint32_t dispatch;
  uint32_t tile;
  uint32_t shards;
} tg_exec_config;
/*   dispatch     : TG_DISPATCH_LISTS (default): each worker polls the counters
 *                  of its own compiled list (schedule, window, notify apply).
 *                  TG_DISPATCH_QUEUE: ready tasks flow through a ticket queue
 *                  (Algorithm 1 EXECUTE_OP on the vertex a COMPLETED_EDGE
 *                  made ready): the decrement that empties a counter makes
 *                  its task ready; the finishing worker keeps one ready
 *                  successor as its next task and pushes the others into the
 *                  next shard in turn (one atomic add on its tail per
 *                  wavefront); a worker that needs work claims a tile of
 *                  tickets of its own shard (one atomic add on the head) and
 *                  waits on each claimed slot; once every sink has run, exit
 *                  sentinels fill every shard.  Needs no co-residency.
 *                  Wavefront and workgroup mappings only.
 *   tile         : queue: tickets claimed per pop (1..64, default 1).
 *   shards       : queue: queue shards (1, 2, 4 or 8; default 8), at most
 *                  the launch's workgroups rounded down to a power of two
 *                  (every shard needs workers that claim from it). */
enum { TG_DISPATCH_LISTS = 1, TG_DISPATCH_QUEUE = 2 };

enum { TG_MAP_WAVE = 1, TG_MAP_WORKGROUP = 2, TG_MAP_GANG = 3 };
enum { TG_SCHED_LIST = 1, TG_SCHED_LEVEL = 2, TG_SCHED_SPREAD = 3, TG_SCHED_COLUMN = 4, TG_SCHED_BALANCED = 5 };

/* ------------------------------------------------------------- status */
const char* tg_status_str(tg_status s);
const char* tg_last_error(void);
/* Library version string; never NULL. */
const char* tg_version(void);

/* Device memory hooks (PyTorch's caching allocator in the Python binding).
 * alloc(bytes, ctx) returns a device pointer or NULL; free_(ptr, ctx).
 * Pass NULL, NULL to return to hipMalloc/hipFree.  Must be called while no
 * graph, batch or server exists. */
tg_status tg_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_)(void* ptr, void* ctx),
                           void* ctx);

/* ------------------------------------------------------------ graphs */

/* Create an empty graph.
 *   mode          : TG_EXPLICIT (events) or TG_IMPLICIT (region requirements).
 *   payload_words : explicit mode: u32 words per task payload, a power of two
 *                   in [64, 65536]; ignored (pass 0) in implicit mode.
 *   index_space   : implicit mode: number of u32 elements of the shared array
 *                   (1 .. 2^36); ignored in explicit mode.
 *   seed          : seed of the initial payloads / initial array.
 * Errors: TG_EINVAL for a bad mode or size, TG_ENOMEM. */
tg_status tg_graph_create(tg_graph* out, uint32_t mode, uint32_t payload_words, uint64_t index_space,
                          uint64_t seed);

/* Explicit mode: add one task predicated on the events preds[0..npreds)
 * (Figure 3 `launch(..., pre)`).  Duplicate events are merged.  Every event
 * must already exist (an index below the current task count), so the graph is
 * acyclic by construction.  *out_event receives the new task's event.
 * Errors: TG_EINVAL (unknown event, wrong mode, NULL out_event), TG_EBUSY
 * after finalise. */
tg_status tg_task_add(tg_graph g, const tg_event* preds, uint32_t npreds, uint32_t mix_rounds,
                      tg_event* out_event);

/* Explicit mode, bulk form: add ntasks tasks whose predecessor lists are
 * preds[pred_ptr[i] .. pred_ptr[i+1]) (pred_ptr has ntasks+1 entries, starting
 * at 0).  Events may refer to tasks of the same call that come earlier.
 * mix_rounds is an array of ntasks values, or NULL to use uniform_rounds for
 * all.  *first_event receives the event of the first added task. */
tg_status tg_task_add_many(tg_graph g, uint32_t ntasks, const uint64_t* pred_ptr, const tg_event* preds,
                           const uint32_t* mix_rounds, uint32_t uniform_rounds, tg_event* first_event);

/* Implicit mode: add one task (next in program order) declaring reqs[0..nreqs).
 * Errors: TG_EINVAL for lo > hi, hi > index_space, an unknown privilege, or a
 * read-write interval overlapping another interval of the same task. */
tg_status tg_task_add_regions(tg_graph g, const tg_region_req* reqs, uint32_t nreqs, uint32_t mix_rounds,
                              tg_event* out_event);

/* Implicit mode, bulk form: task i declares reqs[req_ptr[i] .. req_ptr[i+1]). */
tg_status tg_task_add_regions_many(tg_graph g, uint32_t ntasks, const uint64_t* req_ptr,
                                   const tg_region_req* reqs, const uint32_t* mix_rounds,
                                   uint32_t uniform_rounds, tg_event* first_event);

/* Payload retention of an explicit graph (call before tg_graph_finalize).
 * By default (TG_KEEP_ALL) every task's payload stays in device memory after
 * an execution, so memory is #tasks x payload words.  With TG_KEEP_SINKS a
 * task's payload memory is reused once every task that reads it has
 * finished: compilation gives each task a payload slot (dependence-level
 * order, oldest usable free slot first) and adds, for each reused slot, an
 * anti-dependence edge from every reader of the slot's previous contents to
 * its new owner -- the counters of Algorithm 1 then order the reuse, so the
 * memory is about the payloads alive across two or three dependence levels.
 * Payloads of tasks without successors are kept.  TG_KEEP_NONE reuses those
 * too (only digests are results).  Anti-dependence edges always go to a
 * later dependence level: levels and the critical path are unchanged, and
 * so are digests and kept payloads.  tg_graph_read_payload of a task whose
 * slot was reused gives TG_ESTATE.  TG_EBUSY after finalize, TG_EINVAL for
 * implicit graphs. */
enum { TG_KEEP_ALL = 0, TG_KEEP_SINKS = 1, TG_KEEP_NONE = 2 };
tg_status tg_graph_set_retention(tg_graph g, uint32_t mode);
/* Payload slots of a finalised explicit graph: slot_of[v] (may be NULL; one
 * entry per task), the number of slots and the device bytes they take. */
tg_status tg_graph_payload_slots(tg_graph g, uint32_t* slot_of, uint64_t* nslots, uint64_t* bytes);

/* Compile the graph (Algorithm 1, Compile): merge duplicate predecessors,
 * build the out-edge CSR and in-degree counters, compute the level-ordered
 * schedule, allocate device state.  Implicit mode first infers the dependence
 * DAG on the device (interval-overlap tests in program order).  Idempotent.
 * Blocks until done.  Errors: TG_ENOMEM, TG_EDEVICE. */
tg_status tg_graph_finalize(tg_graph g);

/* Launch one execution of the whole graph on `stream` (Algorithm 1, Execute):
 * counters are reset, so executions repeat with identical results.  Returns
 * without waiting.  cfg may be NULL (the autotuned configuration if one was
 * chosen, else the defaults).  An execution may be launched while the
 * previous one is still running if both use the same stream (stream order
 * serialises them).  Errors: TG_ESTATE if not finalised, TG_EBUSY if a
 * previous execution on another stream has not been waited for. */
tg_status tg_graph_execute(tg_graph g, const tg_exec_config* cfg, void* stream);

/* External pre- and post-condition vertices (Section 4.1): the execution
 * starts only after every hipEvent_t in pre[0..npre) (recorded by the caller,
 * on any stream) has completed, and `post` (a hipEvent_t, may be NULL) is
 * recorded on `stream` when the whole graph has finished, so compiled graphs
 * can be stitched into a larger, dynamically built program.  Otherwise as
 * tg_graph_execute. */
tg_status tg_graph_execute_after(tg_graph g, const tg_exec_config* cfg, void* stream, void* const* pre, uint32_t npre,
                                 void* post);

/* Condition flags: pre- and post-condition vertices that need no stream
 * ordering (Section 4.1: a compiled graph's pre-conditions may be satisfied by
 * the host or by other work at any time, and its post-condition tells whoever
 * waits that the whole graph has finished; Section 4.3: edges between the
 * device and the host).  A flag is one 32-bit word in pinned, coherent host
 * memory mapped for the device, initially 0.
 *   tg_flag_create  : *out receives the flag.  TG_EDEVICE if pinned memory
 *                     cannot be allocated or mapped.
 *   tg_flag_destroy : frees it; no launch in flight may still use it.
 *   tg_flag_set     : host store of value (sequentially consistent).
 *   tg_flag_read    : host load.
 *   tg_flag_wait    : host wait until the flag holds at least value;
 *                     TG_ETIMEOUT after timeout_ms.
 * tg_graph_execute_when: as tg_graph_execute, but the graph's tasks start only
 * once every pre[i] holds at least pre_value[i] (npre <= 8; checked on the
 * device, so the host or a graph running on another stream may meet the
 * condition at any time after the call), and when the whole graph has
 * finished `post` (may be NULL) is set to post_value on the device.  The wait
 * is bounded by the configuration's watchdog interval: if a condition is not
 * met by then the execution is abandoned (no task runs, `post` is left
 * unchanged) and tg_graph_wait reports TG_ETIMEOUT naming the flag.  A launch
 * that waits on a flag holds one wavefront while it waits; its executor
 * occupies the device once the condition holds, so launches that meet the
 * condition should be issued first or fit beside it (same launch shape,
 * workers together within the calibrated capacity), else the residency
 * ordering between streams makes them wait for the waiting launch until its
 * wait times out.  Errors: TG_EINVAL for npre > 8 or NULL flags, else as
 * tg_graph_execute. */
tg_status tg_flag_create(tg_flag* out);
tg_status tg_flag_destroy(tg_flag f);
tg_status tg_flag_set(tg_flag f, uint32_t value);
tg_status tg_flag_read(tg_flag f, uint32_t* value);
tg_status tg_flag_wait(tg_flag f, uint32_t value, uint32_t timeout_ms);
tg_status tg_graph_execute_when(tg_graph g, const tg_exec_config* cfg, void* stream, const tg_flag* pre,
                                const uint32_t* pre_value, uint32_t npre, tg_flag post, uint32_t post_value);

/* Block until the last execution finished; surfaces watchdog aborts
 * (TG_ETIMEOUT) and deferred HIP errors (TG_EDEVICE). */
tg_status tg_graph_wait(tg_graph g);

/* Read results (each waits for an in-flight execution first). */
tg_status tg_graph_num_tasks(tg_graph g, uint64_t* n);
tg_status tg_graph_num_edges(tg_graph g, uint64_t* e);  /* distinct edges executed (reduced ones if reduced) */
tg_status tg_graph_read_digests(tg_graph g, uint32_t* host_out, uint64_t n);  /* n = #tasks */
tg_status tg_graph_read_payload(tg_graph g, tg_event v, uint32_t* host_out, uint32_t n); /* n = payload words */
tg_status tg_graph_read_data(tg_graph g, uint32_t* host_out, uint64_t lo, uint64_t hi);  /* implicit A[lo,hi) */
tg_status tg_graph_checksum(tg_graph g, uint64_t* out);
/* Out-edge CSR of the (inferred or explicit) DAG: row j lists the successors
 * of task j in ascending order.  row_ptr has #tasks+1 entries; col holds up to
 * cap_e entries; *e receives the edge count (TG_ENOMEM if it exceeds cap_e). */
tg_status tg_graph_read_dag(tg_graph g, uint64_t* row_ptr, uint32_t* col, uint64_t cap_e, uint64_t* e);
/* The edges the executor's counters follow, as an out-edge CSR (format as
 * tg_graph_read_dag): the DAG itself, plus the anti-dependence edges of
 * reused payload slots (tg_graph_set_retention), or the reduced DAG after
 * tg_graph_reduce_edges. */
tg_status tg_graph_read_exec_dag(tg_graph g, uint64_t* row_ptr, uint32_t* col, uint64_t cap_e, uint64_t* e);
/* Dependence reduction (Section 5 names transitive reduction as an
 * optimisation of inferred dependences).  tg_reduce_dag: for a DAG given as
 * an out-edge CSR over n vertices whose ids are a topological order (every
 * edge j -> k has j < k; rows may be in any order inside), writes the CSR of
 * the same DAG without every edge j -> k for which some i has edges j -> i
 * and i -> k.  Each dropped edge is implied by a path, so reachability (the
 * order the DAG imposes) is unchanged.  out_row_ptr: n + 1 entries;
 * out_col: capacity row_ptr[n]; rows come out ascending; *out_e = edges kept.
 * Host memory only; cost grows with the sum over edges i -> k of i's
 * in-degree.  TG_EINVAL for an edge that does not go forward.
 * tg_graph_reduce_edges: execute a finalised implicit graph on the two-hop
 * reduction of its last-user DAG (tg_last_user_dag below), which orders the
 * tasks as the inferred DAG does (fewer counter decrements, identical
 * results: an implicit task's inputs come from the shared array, not from
 * its predecessors); tg_graph_read_dag keeps returning the full inferred DAG.
 * *removed (may be NULL) = edges dropped.  TG_EINVAL for explicit graphs,
 * whose predecessor sets are task inputs. */
tg_status tg_reduce_dag(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, uint64_t* out_row_ptr,
                        uint32_t* out_col, uint64_t* out_e);
tg_status tg_graph_reduce_edges(tg_graph g, uint64_t* removed);
/* Last-user dependences of an implicit program (Section 5: the runtime must
 * order conflicting tasks as sequential program order does, and need not
 * record every conflicting pair).  Tasks are visited in program order; each
 * element's history is its last writer and the tasks that read it since.  A
 * task reading an element depends on its last writer; a task writing it
 * depends on the last writer and every reader since.  Every edge joins two
 * conflicting tasks, and every conflicting pair is joined by a path, so the
 * DAG orders the tasks exactly as the inferred conflict DAG does, with a few
 * edges per task instead of one per conflicting pair.
 *   n        : tasks; req_ptr (host, n + 1 u64, req_ptr[0] = 0, ascending)
 *              and reqs (host, req_ptr[n] records) as for
 *              tg_task_add_regions_many.
 *   out_row_ptr : host, n + 1 u64, written: out-edge CSR, rows ascending.
 *   out_col  : host, cap_e u32, written.
 *   *out_e   : edges of the DAG (also on TG_ENOMEM, when it exceeds cap_e).
 * TG_EINVAL for NULL arguments, lo > hi or an unknown privilege.
 * tg_graph_reduce_edges executes the two-hop reduction of this DAG. */
tg_status tg_last_user_dag(uint32_t n, const uint64_t* req_ptr, const tg_region_req* reqs, uint64_t* out_row_ptr,
                           uint32_t* out_col, uint64_t cap_e, uint64_t* out_e);

/* Dependence inference on device-resident requirements (Section 2: tasks
 * declare the data they access and the runtime discovers the dependences;
 * Section 5: the result must equal sequential program order).  The kernels
 * are those of an implicit graph's finalize; the conflict rule is the one
 * stated at the top of this file: tasks j < k conflict iff an interval of j
 * and an interval of k share an element and at least one of the two is
 * read-write, and every conflicting pair is an edge j -> k (no reduction).
 *   ntasks      : tasks in program order (at most 2^31 - 1).
 *   req_ptr     : device, ntasks + 1 u64; task k's requirements are
 *                 reqs[req_ptr[k] .. req_ptr[k+1]); req_ptr[0] = 0,
 *                 non-decreasing, req_ptr[ntasks] = nreqs.
 *   reqs        : device, nreqs tg_region_req records (32 bytes each);
 *                 intervals lie inside [0, index_space); a task's read-write
 *                 interval overlaps none of its own other intervals.
 *   row_ptr     : device, ntasks + 1 u64, written: the out-edge CSR.
 *   col         : device, col_cap u32, written: successors, each row
 *                 ascending.
 *   *num_edges  : host, written: the edge count (also when it exceeds
 *                 col_cap, which returns TG_ENOMEM with col unwritten).
 *   stream      : every kernel runs on it; the call returns when the DAG is
 *                 complete (it waits for the stream, which therefore must not
 *                 be capturing).
 * The caller owns every array.  Scratch device memory (the interval table,
 * buckets, counts, scan partials) is allocated with hipMalloc for the call
 * and freed before it returns.  TG_EINVAL for a bad requirement list (the
 * message names the fault), TG_EDEVICE for a HIP error. */
tg_status tg_infer_dag(uint32_t ntasks, const uint64_t* req_ptr, const tg_region_req* reqs, uint64_t nreqs,
                       uint64_t index_space, uint64_t* row_ptr, uint32_t* col, uint64_t col_cap, uint64_t* num_edges,
                       void* stream);
/* tg_infer_dag for callers that cannot allocate device memory (serving loops
 * that must not call hipMalloc, harnesses that forbid it): same arguments,
 * same result, no hipMalloc, hipFree or allocator call.  Its scratch is one
 * 16 MiB array of device memory in the library's code object, one copy per
 * device, held until the process ends; the call fails with TG_ENOMEM (the
 * message names the array that did not fit) when the requirement list needs
 * more.  The interval table takes 32 bytes per requirement and the row counts
 * 4 bytes per task, so about 400,000 requirements fit (the 65,536-task halo
 * program with 196,480 requirements takes about 9 MiB).  Every call on a
 * device shares that device's array and leaves its contents behind; each call
 * clears what it reads before writing it.  Calls from this process on one
 * device are serialised by a lock; calls from two processes use two copies.
 * Outputs are unspecified after an error other than TG_ENOMEM for col_cap. */
tg_status tg_infer_dag_noalloc(uint32_t ntasks, const uint64_t* req_ptr, const tg_region_req* reqs, uint64_t nreqs,
                               uint64_t index_space, uint64_t* row_ptr, uint32_t* col, uint64_t col_cap,
                               uint64_t* num_edges, void* stream);

/* Times of the last finalize (host compile, device inference) and of the last
 * execution measured with HIP events, in milliseconds (0 when not measured). */
tg_status tg_graph_timings(tg_graph g, double* compile_ms, double* infer_ms, double* exec_ms);
tg_status tg_graph_destroy(tg_graph g);

/* ------------------------------------------------------------ batches */

/* Compile n finalised graphs of either mode into one persistent launch
 * (graphs stay independent; each keeps its own results).  cfg may be NULL. */
tg_status tg_batch_create(tg_batch* out, const tg_graph* graphs, uint32_t n, const tg_exec_config* cfg);
tg_status tg_batch_execute(tg_batch b, void* stream);
tg_status tg_batch_wait(tg_batch b);
/* Device time of the last batch execution (HIP events), in milliseconds. */
tg_status tg_batch_time_ms(tg_batch b, double* ms);
/* Executor-kernel durations of the batch's most recent launches (as
 * tg_graph_kernel_times). */
tg_status tg_batch_kernel_times(tg_batch b, double* ms_out, uint32_t n, uint32_t* got);
/* Give every task of every graph of the batch `uniform_rounds` mix rounds. */
tg_status tg_batch_set_rounds(tg_batch b, uint32_t uniform_rounds);
/* Launch shape of the batch (workers = the actual count), its task count,
 * and the host time spent building its current layout: plan_ms for the
 * schedule and task records, build_ms for all of it including the upload
 * (Algorithm 1, Compile).  Any output pointer may be NULL. */
tg_status tg_batch_info(tg_batch b, tg_exec_config* cfg, uint64_t* tasks, double* plan_ms, double* build_ms);
/* Edges of the batch's layout signalled with a counter atomic per launch
 * (Algorithm 1 COMPLETED_EDGE): all executed edges, less those between
 * consecutive entries of one worker's list, which the list dispatch does not
 * count (their order follows from the list) unless the workers are gangs
 * (whose members signal every edge, once each).  TG_EINVAL for NULL
 * arguments. */
tg_status tg_batch_signalled_edges(tg_batch b, uint64_t* edges);
/* Autotuner for a batch (as tg_graph_autotune); keeps the fastest layout. */
tg_status tg_batch_autotune(tg_batch b, uint32_t reps, tg_exec_config* best, double* best_ms);
tg_status tg_batch_destroy(tg_batch b);

/* Residency of the persistent executor.  Every worker of a launch must be
 * resident at the same time, so the library never launches more workers than
 * a probe launch of the executor kernel has shown to be co-resident.
 *   blocks_per_cu : the runtime's occupancy estimate (an upper bound);
 *   cus           : compute units of the current device;
 *   resident      : if not NULL, the calibrated number of co-resident
 *                   workers (measured once per device and kernel variant). */
tg_status tg_exec_occupancy(uint32_t mapping, uint32_t wg_waves, uint32_t* blocks_per_cu, uint32_t* cus,
                            uint32_t* resident);
/* Workers of the graph's last launch and, for a diagnostic launch (diag=1),
 * how many of them started. */
tg_status tg_graph_exec_info(tg_graph g, uint32_t* workers, uint32_t* started);
/* Host-only model of a launch of graphs[0..ngraphs) together (one graph
 * alone, or a batch), no GPU needed: compiles the worker layout for nworkers
 * workers with the given schedule (0 = default) and steps the same
 * ready-window loop as the kernels in a seeded order.  order (total #tasks
 * entries) receives the execution order as (graph index << 32 | event),
 * *executed the number of tasks run; TG_ETIMEOUT if the layout would
 * deadlock.  If makespan and bound are not NULL, the layout is also run in a
 * timed model (each task takes the cost the scheduler estimates for it):
 * *makespan is its finishing time and *bound the lower bound
 * max(longest path, total cost / workers), both in the same cost units. */
tg_status tg_emulate_schedule(const tg_graph* graphs, uint32_t ngraphs, uint32_t nworkers, uint32_t window,
                              uint32_t schedule, uint64_t seed, uint64_t* order, uint64_t* executed, uint64_t* makespan,
                              uint64_t* bound);
/* Host-only model of the ready-queue dispatch (TG_DISPATCH_QUEUE) over
 * graphs[0..ngraphs): nworkers workers with the kernels' steps (a claim of
 * `tile` tickets by one atomic add on the head of the worker's shard, then a
 * wait on each claimed slot; pushes of the ready successors by one atomic
 * add on the tail of the next shard in turn, one ready successor kept per
 * completion; sinks counted by workers whose next slot is empty, and exit
 * sentinels pushed into every shard by the count that completes the total),
 * interleaved in a seeded order at every access to shared state.  shards
 * must be a power of two in 1..8 and tile in 1..64 (TG_EINVAL otherwise).  order (total #tasks entries) receives the
 * execution order as (graph index << 32 | event); TG_ETIMEOUT if the model
 * does not terminate. */
tg_status tg_emulate_queue(const tg_graph* graphs, uint32_t ngraphs, uint32_t nworkers, uint32_t shards, uint32_t tile,
                           uint64_t seed, uint64_t* order, uint64_t* executed);
/* Host-only model of a gang launch (mapping 3, Algorithm 1 EXECUTE_OP with
 * one task per gang of workgroups) over graphs[0..ngraphs): ngangs lists
 * compiled with `schedule` (0 = default), and `gang` members per list that
 * each scan, take and finish their share on their own, in a seeded
 * interleaving; a counter starts at in-degree x gang and each member
 * decrements every out-edge once.  Checks that a member takes a task only
 * after every member of each predecessor finished it and that every member
 * runs each entry of its list exactly once.  elide != 0 models the lists'
 * in-list edge elision, which gang launches do not use (a member could then
 * run ahead of the others; the check reports it).  *executed = shares
 * finished (total #tasks x gang on success); TG_ETIMEOUT if the members get
 * stuck, TG_EINVAL for a violated check or arguments out of range (window
 * 1..64, ngangs >= 1, gang 1..32). */
tg_status tg_emulate_gang(const tg_graph* graphs, uint32_t ngraphs, uint32_t ngangs, uint32_t gang, uint32_t window,
                          uint32_t schedule, uint64_t seed, uint32_t elide, uint64_t* executed);
/* After a diagnostic launch (diag=1) of the graph on its own: per task (by
 * event) the pending in-edge counter (with gangs, every in-edge counts once
 * per gang member), the number of times it ran, its worker
 * and its entry in that worker's list; optionally (wprog != NULL, nworkers =
 * the launch's worker count) how many list entries each worker finished. */
tg_status tg_graph_debug_state(tg_graph g, uint32_t* pending, uint32_t* execs, uint32_t* owner, uint32_t* entry,
                               uint32_t* wprog, uint32_t nworkers);
/* After a diagnostic launch: per task (by event) the device clock at its
 * start and at the end of its edge signals (2 u64 per task, 100 MHz ticks,
 * 0 if it never ran); optionally per worker [first scan, last scan, scans,
 * reserved]. */
tg_status tg_graph_debug_times(tg_graph g, uint64_t* task_times, uint64_t* worker_stamps, uint32_t nworkers);

/* Device time of the executor kernel alone in the last execution (the
 * counter reset before it excluded), in milliseconds. */
tg_status tg_graph_kernel_ms(tg_graph g, double* kernel_ms);
/* Executor-kernel durations (ms, HIP events on the launch stream) of the
 * graph's most recent launches, oldest first: up to n (at most 64) values
 * into ms_out, count in *got.  Waits for the last execution. */
tg_status tg_graph_kernel_times(tg_graph g, double* ms_out, uint32_t n, uint32_t* got);
/* Give every task of a compiled graph `uniform_rounds` mix rounds (the
 * schedule is kept; only the task records are rewritten). */
tg_status tg_graph_set_rounds(tg_graph g, uint32_t uniform_rounds);

/* Autotuner: time the candidate launch configurations (wavefront or
 * workgroup or gang per task, worker and gang counts, workgroup sizes,
 * schedules, doorbell mode, the ready queue) on
 * this graph, reps executions each, and keep the fastest as the graph's
 * default (used when tg_graph_execute gets cfg == NULL).  Results never
 * depend on the configuration.  *best receives the chosen one; best_ms its
 * mean kernel time. */
tg_status tg_graph_autotune(tg_graph g, uint32_t reps, tg_exec_config* best, double* best_ms);

/* Roofline probes (run on the current device, synchronous). */
enum {
  TG_PROBE_MIX_RATE = 1,         /* word-rounds/s of the body's mix, no dependences */
  TG_PROBE_COPY_BW = 2,          /* bytes/s read + written by a streaming copy */
  TG_PROBE_ATOMIC_DISTINCT = 3,  /* device-scope u32 atomics/s on distinct addresses */
  TG_PROBE_ATOMIC_CONTENDED = 4, /* device-scope u32 atomics/s on one address */
  TG_PROBE_LAUNCH_RATE = 5,      /* empty kernel launches/s, back to back */
  TG_PROBE_HANDOFF_NS = 6,       /* ns of one dependent hop between wavefronts on two
                                    neighbouring XCDs: see the signal, load the 1 KB
                                    payload, store one, drain the stores, signal with
                                    one atomic (the per-level floor of a dependence
                                    chain) */
  TG_PROBE_HANDOFF_SAME_XCD_NS = 7,  /* the same hop between two CUs of one XCD */
  TG_PROBE_HANDOFF_FAR_XCD_NS = 8,   /* ... between XCDs in the two halves of the package */
  TG_PROBE_HANDOFF_L2_NS = 9         /* ... within one XCD, the payload loaded and stored
                                        through the XCD's L2 (L1 bypassed) instead of at
                                        device scope; the signal stays device scope */
};
tg_status tg_probe(uint32_t kind, double* value);

/* ------------------------------------------------------------ serving */

/* A server admits submitted graphs while their device memory fits
 * budget_bytes, groups the admitted ones (at most max_batch per launch) into
 * persistent launches on up to `slots` streams (1..4; 0 = 4), and retires
 * launches as they finish: continuous batching.  Requests arriving while
 * others run are admitted as soon as a slot and memory free up.  On
 * completion a request's digests are copied to the host (tg_graph_read_digests
 * and tg_graph_checksum keep working) and its device memory is released.
 * A request larger than the whole budget fails with TG_ENOMEM.  With more than
 * one slot, requests of 65,536 tasks or more run in slot 0 only (which also
 * takes smaller ones while no large one waits), so small requests do not share
 * a launch with graphs that keep it busy for long.  With the ready queue
 * (tg_server_configure) a request completes as soon as its graph has, while
 * its launch may still run other graphs. */
tg_status tg_server_create(tg_server* out, uint64_t budget_bytes, uint32_t slots, uint32_t max_batch);
/* Launch configuration of the batches a server issues from now on (Section
 * 4.1: compiled graphs issued dynamically).  Default: TG_DISPATCH_QUEUE with
 * one wavefront per task, tile 1, 8 shards and the co-resident workers
 * divided over the slots.  With the ready queue a batch needs no host
 * schedule: each graph's compiled form (its predecessor and successor
 * lists, counter reset values, rounds, requirements and sources, packed at
 * finalize) is uploaded once when the graph is admitted, and one device
 * kernel builds the batch's task records from them; the slot keeps its
 * buffers for the next batch.  TG_DISPATCH_LISTS plans per-worker lists and
 * builds the records on the host for every batch (mapping, workers,
 * schedule and window apply).  Gangs are refused (TG_EINVAL). */
tg_status tg_server_configure(tg_server srv, const tg_exec_config* cfg);
/* Non-blocking.  g must be compiled (finalised) and not executing; the caller
 * keeps ownership and must not touch g until the ticket is waited for.  A
 * graph whose request has not finished cannot be submitted again: TG_EBUSY. */
tg_status tg_server_submit(tg_server srv, tg_graph g, uint64_t* ticket);
/* Blocks until the request finished; returns its status and the steady-clock
 * times (ns) of submission, admission and completion.  Each ticket is waited
 * for once. */
tg_status tg_server_wait(tg_server srv, uint64_t ticket, uint64_t* submit_ns, uint64_t* admit_ns, uint64_t* done_ns);
/* Totals so far: tasks finished, launches, peak admitted bytes; phase_ms (9
 * doubles, may be NULL): host time of the serving threads building layouts
 * (device buffers, schedule, upload), issuing launches and retiring finished
 * launches (results copied back, buffers released); the device time of all
 * launches (HIP events around each); and, inside the host time, the time
 * spent planning schedules and records, in the device-memory allocator
 * (hooks or hipMalloc/hipFree), in host-device copies, and (records built on
 * the device) preparing the admitted graphs' device buffers and setting up
 * the layout's buffers, tables and kernels. */
tg_status tg_server_stats(tg_server srv, uint64_t* tasks_done, uint64_t* launches, uint64_t* peak_bytes,
                          double* phase_ms);
/* Finishes all submitted work, then stops the server thread. */
tg_status tg_server_destroy(tg_server srv);

/* ------------------------------------------------------- comparators */

/* Plain comparators of the same graph: one kernel launch per task in creation
 * order on `stream` (mode 1); replay of a hipGraph with one kernel node per
 * task and one dependency per edge (mode 2); replay of the mode-1 launch
 * sequence captured from a stream into a hipGraph (mode 3).  Each hipGraph is
 * built and instantiated on the first call and cached until the graph's
 * layout changes.  Results are identical to tg_graph_execute. */
enum { TG_CMP_PER_TASK = 1, TG_CMP_HIPGRAPH = 2, TG_CMP_HIPGRAPH_CAPTURED = 3 };
tg_status tg_graph_execute_comparator(tg_graph g, uint32_t mode, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TASKGRAPH_H */
