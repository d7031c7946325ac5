// Persistent task-DAG executor for gfx950 (MI355X).
//
// Algorithm 1 of the paper compiles a fixed graph into per-resource worker
// actors: each vertex keeps an atomic counter of pending in-edges, a finished
// vertex sends one COMPLETED_EDGE per out-edge (an atomic decrement), and a
// vertex runs once its counter reaches zero.  Here a worker is a wavefront
// (mapping 1) or a workgroup (mapping 2) of one persistent launch.
//
//  * Event subsystem: one u32 counter per task in HBM, reset from the
//    in-degree before each execution and decremented once per edge with a
//    device-scope atomic.  A task is ready exactly when its counter is 0.
//  * Ready subsystem: the compiler hands every worker its own list of
//    positions in dependence-level order.  A worker polls the counters of
//    the next `window` (<= 64) unfinished positions of its list with one
//    lane per position, compacts the ready ones with a wave ballot, runs them
//    in list order and slides the window past the finished prefix.  No
//    address is shared between workers except the counters of real edges,
//    so there is no contended queue head or tail (a single-address device
//    atomic costs about 11 ns on this part; distinct addresses sustain
//    about 27 G atomics/s).
//  * Publication: payload and array writes use device-coherent (sc1)
//    stores; before the first out-edge decrement the worker waits for all
//    its stores to complete (s_waitcnt vmcnt(0)).  Readers load with sc1.
//    This avoids the L2 write-back that an agent-scope release fence issues
//    on gfx950, which costs about 13 ns per publication device-wide.
//  * Every wait is bounded: a worker whose wait has lasted the watchdog
//    interval aborts the launch only if no worker anywhere has started a
//    task for that long (workers publish a device-wide progress stamp, at
//    most once per 1/16 of the interval each); every other worker returns
//    when it sees the abort flag.  A long critical path that keeps most
//    workers idle therefore never trips the watchdog while it advances.
#include "tg_internal.h"

namespace tg {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kSC1 = 16;  // buffer cache policy: device-scope coherent access

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, nbytes, 0x00020000);
}

// Wait until every outstanding vector memory operation of this wave has
// completed; the memory clobber keeps the compiler from moving memory
// operations across it.
__device__ __forceinline__ void vm_drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Read-only tables (records, graph table, predecessor addresses, requirement
// lists) are read through the constant address space so that wave-uniform
// accesses become scalar loads.
// (The host compilation pass sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using cptr = const T __attribute__((address_space(4)))*;
#else
template <class T>
using cptr = const T*;
#endif
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)p;
}
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint32_t ld_coherent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- hashing

__device__ __forceinline__ uint64_t sm64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// low 32 bits of sm64(key ^ idx), key = sm64(seed ^ (stream << 32))
__device__ __forceinline__ uint32_t h32k(uint64_t key, uint64_t idx) { return (uint32_t)sm64(key ^ idx); }

template <class V>
__device__ __forceinline__ V mix_rounds(V x, uint32_t R) {
  for (uint32_t r = 0; r < R; ++r) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    x = x * 0x9E3779B1u + 0x7F4A7C15u;
  }
  return x;
}

// Wrap-around sum over the 64 lanes (all active), returned wave-uniform.
// Cross-lane moves within each 16-lane row use DPP (swap neighbours, swap
// pairs, mirror each half-row, mirror the row); the four row sums are then
// read with readlane.  No LDS round trip: this sits between a task's payload
// store and its digest store, on the task's critical path.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
         __builtin_amdgcn_readlane(v, 48);
}

// ------------------------------------------------------------------ teams

// A team is the set of lanes that executes one task: one wavefront, one
// workgroup, or (gang) the same lane slot of several workgroups on different
// CUs.  t / size() index the lanes of this wavefront or workgroup: sum()
// returns the wrap-around sum of v over them to every lane and sync() is
// their barrier.  wt() / ws() index the task's work items over the whole
// team (equal to t / size() except in a gang).
struct WaveTeam {
  uint32_t t;
  static constexpr uint32_t S = 64;
  __device__ __forceinline__ uint32_t size() const { return 64; }
  __device__ __forceinline__ uint32_t wt() const { return t; }
  __device__ __forceinline__ uint32_t ws() const { return 64; }
  __device__ __forceinline__ uint32_t sum(uint32_t v) const { return wave_sum(v); }
  __device__ __forceinline__ void sync() const {}
  __device__ __forceinline__ bool leader() const { return t == 0; }
};

struct BlockTeam {
  uint32_t t, n;
  uint32_t* lds;  // >= 17 words
  __device__ __forceinline__ uint32_t size() const { return n; }
  __device__ __forceinline__ uint32_t wt() const { return t; }
  __device__ __forceinline__ uint32_t ws() const { return n; }
  __device__ __forceinline__ void sync() const { __syncthreads(); }
  __device__ __forceinline__ bool leader() const { return t == 0; }
  __device__ uint32_t sum(uint32_t v) const {
    v = wave_sum(v);
    const uint32_t w = t >> 6;
    __syncthreads();
    if ((t & 63) == 0) lds[w] = v;
    __syncthreads();
    uint32_t s = 0;
    for (uint32_t i = 0; i < (n >> 6); ++i) s += lds[i];
    return s;
  }
};

// One workgroup (member m of G) of a gang: reductions and barriers stay
// inside the workgroup, work items are split over all G workgroups.
struct GangTeam : BlockTeam {
  uint32_t m, G;
  __device__ __forceinline__ uint32_t wt() const { return m * n + t; }
  __device__ __forceinline__ uint32_t ws() const { return G * n; }
  __device__ __forceinline__ bool leader() const { return m == 0 && t == 0; }
};

// ----------------------------------------------------------------- record

__device__ __forceinline__ uint32_t rl(uint32_t v, uint32_t k) { return __builtin_amdgcn_readlane(v, k); }

// A task record as one team holds it: every wavefront loads the 128-byte
// record with one coalesced load (lane i: dword i % 32) and reads the scalar
// fields out with readlane.  succ0 is the successor this team index signals
// first (index t), fetched together with the record so that no load stands
// between the payload store and the edge signals.
struct Rec {
  uint32_t v;
  uint64_t out;
  uint32_t tid, graph, pred_beg, npred, succ_beg, nsucc, rounds, nreq;
  uint32_t succ0;
  uint32_t* digest;  // the graph's digest array
};

// This lane's dword of the record at `pos`.  Records are read-only while a
// launch runs, so a plain (cached) load is enough.
__device__ __forceinline__ uint32_t rec_dword(const ExecParams& P, uint32_t pos, uint32_t lane) {
  return reinterpret_cast<const uint32_t*>(P.rec + pos)[lane & 31u];
}

template <class Team>
__device__ __forceinline__ void unpack_rec(const Team& tm, const ExecParams& P, uint32_t v, Rec& r) {
  const uint32_t lane = tm.t & 63u;
  r.v = v;
  r.out = (uint64_t)rl(r.v, kDwOut) | ((uint64_t)rl(r.v, kDwOut + 1) << 32);
  r.tid = rl(r.v, kDwTid);
  r.graph = rl(r.v, kDwGraph);
  r.pred_beg = rl(r.v, kDwPredBeg);
  r.npred = rl(r.v, kDwNpred);
  r.succ_beg = rl(r.v, kDwSuccBeg);
  r.nsucc = rl(r.v, kDwNsucc);
  r.rounds = rl(r.v, kDwRounds);
  r.nreq = rl(r.v, kDwNreq);
  const uint32_t inl = __shfl(r.v, (int)(kDwSucc + (lane & (kInSucc - 1))), 64);
  const uint32_t j = tm.t;
  r.succ0 = 0;
  if (j < r.nsucc) r.succ0 = j < kInSucc ? inl : P.succ_pos[r.succ_beg + j];
}

// Payload address of predecessor j (j wave-uniform).
__device__ __forceinline__ uint64_t pred_at(const ExecParams& P, const Rec& r, uint32_t j) {
  if (j < kInPred) return (uint64_t)rl(r.v, kDwPred + 2 * j) | ((uint64_t)rl(r.v, kDwPred + 2 * j + 1) << 32);
  return as_const(P.pred_addr)[r.pred_beg + j];
}

// ------------------------------------------------------------------ bodies

template <int VEC>
struct VecT;
template <>
struct VecT<1> { typedef uint32_t T; };
template <>
struct VecT<2> { typedef u32x2 T; };
template <>
struct VecT<4> { typedef u32x4 T; };

template <int VEC>
__device__ __forceinline__ typename VecT<VEC>::T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  if constexpr (VEC == 4) return __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, kSC1);
  else if constexpr (VEC == 2) return __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, kSC1);
  else return __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, kSC1);
}
template <int VEC>
__device__ __forceinline__ void buf_store(typename VecT<VEC>::T v, __amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  if constexpr (VEC == 4) __builtin_amdgcn_raw_buffer_store_b128(v, r, byte_off, 0, kSC1);
  else if constexpr (VEC == 2) __builtin_amdgcn_raw_buffer_store_b64(v, r, byte_off, 0, kSC1);
  else __builtin_amdgcn_raw_buffer_store_b32(v, r, byte_off, 0, kSC1);
}

template <int VEC>
__device__ __forceinline__ uint32_t elem(typename VecT<VEC>::T v, int i) {
  if constexpr (VEC == 1) return v;
  else return v[i];
}

// Explicit body over words k = k0, k0 + VEC*S, ... handled VEC at a time.
// The chunk loop and the mix-round loop have wave-uniform trip counts (n,
// the team size and R are uniform), so both run under scalar loop control;
// lanes whose chunk lies past the payload (a team wider than n / VEC) only
// skip the loads and the store.
template <int VEC, class Team>
__device__ __forceinline__ uint32_t explicit_words(const Team& tm, const ExecParams& P, const Rec& r,
                                                   const GraphEnt& G) {
  typedef typename VecT<VEC>::T V;
  const uint32_t n = G.n, S = tm.ws();
  const uint32_t nbytes = n * 4u;
  const uint32_t npred = r.npred, R = r.rounds, tid = r.tid;
  const __amdgpu_buffer_rsrc_t wr = make_rsrc((const void*)r.out, nbytes);
  const uint32_t step = VEC * S;
  const uint32_t chunks = uni((n + step - 1u) / step);
  uint32_t dsum = 0;
  for (uint32_t c = 0; c < chunks; ++c) {
    const uint32_t k0 = c * step + tm.wt() * VEC;
    const bool valid = k0 < n;
    V acc = V(0);
    if (valid) {
      if (npred == 0) {
        // source: initial payload from the graph seed
        if constexpr (VEC == 1) {
          acc = h32k(G.key1, ((uint64_t)tid << 16) | k0);
        } else {
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc[i] = h32k(G.key1, ((uint64_t)tid << 16) | (k0 + i));
        }
      } else {
        // groups of up to five predecessors, each group's loads issued
        // together: one memory round trip per group, not per predecessor
        uint32_t j = 0;
        while (j < npred) {
          const uint32_t m = npred - j;  // wave-uniform
          const __amdgpu_buffer_rsrc_t r0 = make_rsrc((const void*)pred_at(P, r, j), nbytes);
          if (m >= 5) {
            V a0 = buf_load<VEC>(r0, k0 * 4);
            V a1 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 1), nbytes), k0 * 4);
            V a2 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 2), nbytes), k0 * 4);
            V a3 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 3), nbytes), k0 * 4);
            V a4 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 4), nbytes), k0 * 4);
            acc += ((a0 + a1) + (a2 + a3)) + a4;
            j += 5;
          } else if (m == 4) {
            V a0 = buf_load<VEC>(r0, k0 * 4);
            V a1 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 1), nbytes), k0 * 4);
            V a2 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 2), nbytes), k0 * 4);
            V a3 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 3), nbytes), k0 * 4);
            acc += (a0 + a1) + (a2 + a3);
            j += 4;
          } else if (m == 3) {
            V a0 = buf_load<VEC>(r0, k0 * 4);
            V a1 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 1), nbytes), k0 * 4);
            V a2 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 2), nbytes), k0 * 4);
            acc += (a0 + a1) + a2;
            j += 3;
          } else if (m == 2) {
            V a0 = buf_load<VEC>(r0, k0 * 4);
            V a1 = buf_load<VEC>(make_rsrc((const void*)pred_at(P, r, j + 1), nbytes), k0 * 4);
            acc += a0 + a1;
            j += 2;
          } else {
            acc += buf_load<VEC>(r0, k0 * 4);
            j += 1;
          }
        }
      }
    }
    V x = mix_rounds<V>(acc ^ tid, R);
    if (valid) {
      buf_store<VEC>(x, wr, k0 * 4);
#pragma unroll
      for (int i = 0; i < VEC; ++i) dsum += elem<VEC>(x, i) * (2u * (k0 + i) + 1u);
    }
  }
  return dsum;
}

// Returns the digest part of this wavefront / workgroup (the whole digest
// unless the team is a gang).
template <class Team>
__device__ __forceinline__ uint32_t body_explicit(const Team& tm, const ExecParams& P, const Rec& r,
                                                  const GraphEnt& G) {
  const uint32_t n = G.n, S = tm.ws();
  uint32_t dsum;
  if (n >= 4 * S) dsum = explicit_words<4>(tm, P, r, G);
  else if (n >= 2 * S) dsum = explicit_words<2>(tm, P, r, G);
  else dsum = explicit_words<1>(tm, P, r, G);
  return tm.sum(dsum);
}

// Elements t, t + S, t + 2S, t + 3S of p[0, len) (0 past the end).
__device__ __forceinline__ u32x4 load4(const uint32_t* p, uint32_t t, uint32_t S, uint64_t len) {
  u32x4 x;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t o = t + (uint64_t)k * S;
    x[k] = o < len ? ld_coherent(p + o) : 0u;
  }
  return x;
}

// Returns the digest part of this wavefront / workgroup (the whole digest
// unless the team is a gang).  Every workgroup of a gang sums all read-only
// elements itself; the read-write elements are split over the gang.
template <class Team>
__device__ __forceinline__ uint32_t body_implicit(const Team& tm, const ExecParams& P, const Rec& r,
                                                  const GraphEnt& G) {
  const cptr<ReqDev> rq = as_const((const ReqDev*)r.out);
  uint32_t* A = G.data;
  // read-only elements: their wrap sum c
  uint32_t part = 0;
  for (uint32_t i = 0; i < r.nreq; ++i) {
    const ReqDev q = rq[i];
    if (q.priv != 1) continue;
    for (uint64_t e = q.lo + tm.t; e < q.hi; e += tm.size()) part += ld_coherent(A + e);
  }
  const uint32_t key = uni(tm.sum(part) ^ r.tid);
  const uint32_t R = r.rounds;
  const uint32_t S = tm.ws(), wt = tm.wt();
  uint32_t dsum = 0;
  for (uint32_t i = 0; i < r.nreq; ++i) {
    const ReqDev q = rq[i];
    if (q.priv != 2) continue;
    const uint64_t len = q.hi - q.lo;
    uint32_t* const a = A + q.lo;
    // four elements per lane per chunk; the chunk loop and the mix-round
    // loop are wave-uniform, lanes past the end skip loads and stores; the
    // next chunk's loads are issued before this chunk's mix
    const uint64_t step = 4 * (uint64_t)S;
    u32x4 x = load4(a, wt, S, len);
    for (uint64_t base = 0; base < len; base += step) {
      const u32x4 y = base + step < len ? load4(a + base + step, wt, S, len - base - step) : u32x4{0, 0, 0, 0};
      x = mix_rounds<u32x4>(x ^ key, R);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t o = base + wt + (uint64_t)k * S;
        if (o < len) {
          st_coherent(a + o, x[k]);
          dsum += x[k] * (2u * (q.rw_base + (uint32_t)o) + 1u);
        }
      }
      x = y;
    }
  }
  return tm.sum(dsum);
}

// Run the task at `pos`; v is this lane's dword of its record.  Returns the
// digest part of this wavefront / workgroup; run_task also stores it.
template <class Team>
__device__ __forceinline__ uint32_t run_body(const Team& tm, const ExecParams& P, uint32_t pos, uint32_t v, Rec& r) {
  unpack_rec(tm, P, v, r);
  const GraphEnt G = as_const(P.gtab)[r.graph];
  r.digest = G.digest;
  if (P.tstamp && tm.leader()) P.tstamp[2 * pos] = __builtin_amdgcn_s_memrealtime();
  const uint32_t d = G.mode == 1 ? body_explicit(tm, P, r, G) : body_implicit(tm, P, r, G);
  if (P.execs && tm.leader()) __hip_atomic_fetch_add(P.execs + pos, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return d;
}

template <class Team>
__device__ __forceinline__ void run_task(const Team& tm, const ExecParams& P, uint32_t pos, uint32_t v, Rec& r) {
  const uint32_t d = run_body(tm, P, pos, v, r);
  // device-coherent, so it is in memory once the team's stores are drained
  // (a graph's digests may be read while its launch still runs)
  if (tm.leader()) st_coherent(r.digest + r.tid, d);
}

// Signal every out-edge of a finished task (COMPLETED_EDGE).
template <class Team>
__device__ __forceinline__ void signal_edge(const ExecParams& P, uint32_t dst) {
  if (P.notify) {
    // COMPLETED_EDGE plus, for the edge that empties a counter, the message
    // that starts the task at its owner: the owner's doorbell is rung only
    // after the decrement has been performed (its old value has returned).
    const uint32_t old = __hip_atomic_fetch_sub(P.cnt + dst, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((old & kPendingMask) == 1u)
      __hip_atomic_fetch_add(P.bell + P.owner[dst] * kBellStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_fetch_sub(P.cnt + dst, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <class Team>
__device__ __forceinline__ void complete_edges(const Team& tm, const ExecParams& P, const Rec& r) {
  vm_drain();  // this lane's payload stores are complete
  tm.sync();   // ... and so are every other lane's of the team
  if (tm.t < r.nsucc) signal_edge<Team>(P, r.succ0);
  for (uint32_t j = tm.t + tm.size(); j < r.nsucc; j += tm.size()) signal_edge<Team>(P, P.succ_pos[r.succ_beg + j]);
}

// A launch behind a pre-condition wait (k_wait_flags) does nothing if the
// wait gave up: the wait raised the abort flag, which the reset before it
// had cleared.
__device__ __forceinline__ bool gate_closed(const ExecParams& P) {
  return P.gated && uni(ld_coherent(&P.ctrl->abort)) != 0u;
}

// ------------------------------------------------------------ worker loop

constexpr uint32_t kExit = 0xFFFFFFFFu;

// Per-worker scheduling state; every field holds the same value in all
// lanes of the wave that runs the state machine.
struct WorkerState {
  uint32_t worker, wb, wcnt;  // list of positions [wb, wb + wcnt)
  uint32_t h;                 // first unfinished list entry
  uint64_t done;              // bit i: entry h + i already taken
  uint64_t pend;              // ready entries found by the last scan, not yet taken
  uint32_t seen;              // last doorbell value read
  uint32_t spins;             // consecutive empty polls
  uint64_t last;              // time of the last task taken (realtime counter)
  uint64_t pub;               // time this worker last published Ctrl::progress
  bool rescan;                // the window must be scanned before waiting
  uint32_t pf_pos;            // position whose record dword is held in pf_v
  uint32_t pf_v;              // per lane: dword lane % 32 of that record
};

__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

// One poll of the ready window: every lane reads one counter and a ballot
// collects the ready entries.  The record of the oldest unfinished entry,
// the likeliest next task, is fetched in the same round trip (once per
// entry), so a task that becomes ready while its worker waits for it starts
// without another dependent load.
__device__ __forceinline__ uint64_t ready_scan(uint32_t lane, const ExecParams& P, WorkerState& w) {
  const uint32_t head = w.wb + w.h;
  if (head != w.pf_pos) {
    w.pf_v = rec_dword(P, head, lane);
    w.pf_pos = head;
  }
  const uint32_t idx = w.h + lane;
  const bool valid = lane < P.window && idx < w.wcnt && !((w.done >> lane) & 1ull);
  uint32_t c = 1u;
  if (valid) c = ld_coherent(P.cnt + w.wb + idx);
  // an entry marked kAfterPrev also needs the entry before it taken (entry
  // h - 1 is finished; this worker runs its tasks one after another)
  const bool prev_taken = lane == 0u || ((w.done >> (lane - 1u)) & 1ull);
  return uni64(__ballot(valid && (c & kPendingMask) == 0u && (!(c & kAfterPrev) || prev_taken)));
}

// Global progress: a worker that takes a task publishes the time (atomic
// max on one word), at most once per progress_ticks, so the word is written
// rarely however many tasks run.
__device__ __forceinline__ void publish_progress(const ExecParams& P, WorkerState& w, uint64_t now, bool lead) {
  if (now - w.pub < P.progress_ticks) return;
  w.pub = now;
  if (lead) __hip_atomic_fetch_max(&P.ctrl->progress, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True when nothing has progressed for the watchdog interval: neither this
// wait (which began at `since`) nor any worker's published task start is
// more recent than watchdog_ticks before `now`.  Clocks read by different
// waves may differ slightly, so a stamp later than `now` counts as `now`.
__device__ __forceinline__ bool stalled(const ExecParams& P, uint64_t since, uint64_t now) {
  if (now - since <= P.watchdog_ticks) return false;
  uint64_t g = __hip_atomic_load(&P.ctrl->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  g = ((uint64_t)uni((uint32_t)(g >> 32)) << 32) | uni((uint32_t)g);
  if (g > now) return false;
  return now - g > P.watchdog_ticks;
}

// Back-off after `spins` consecutive empty polls, in naps of 128 cycles: one
// nap for the first 64 polls, then idle_sleep naps, doubling after every
// further 64 empty polls up to 32 x idle_sleep (at most 256 naps, 14 us).  A
// worker waiting for a quick hand-off polls again at once; one waiting behind
// a long task soon polls only every few microseconds, and so stops taking
// issue slots from the waves on its SIMD that run tasks (measured on 4096
// graphs of log-normal mix rounds: 1523 ms with a fixed 2-nap back-off,
// 1366 ms with 64 naps).
__device__ __forceinline__ void idle_nap(const ExecParams& P, uint32_t spins) {
  uint32_t nap = 1;
  if (spins >= 64) nap = min(P.idle_sleep << min((spins >> 6) - 1u, 5u), 256u);
  for (uint32_t i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(2);
}

// One empty poll: back off, and every 64 polls check the abort flag and the
// watchdog.  Returns false when the worker must stop.
__device__ __forceinline__ bool idle_step(const ExecParams& P, WorkerState& w, uint32_t lane) {
  ++w.spins;
  idle_nap(P, w.spins);
  if ((w.spins & 63u) != 0u) return true;
  if (uni(ld_coherent(&P.ctrl->abort)) != 0u) return false;
  const uint64_t now = __builtin_amdgcn_s_memrealtime();
  if (stalled(P, w.last, now) || (P.spin_limit != 0u && w.spins >= P.spin_limit)) {
    if (lane == 0) {
      const uint32_t prev = __hip_atomic_fetch_add(&P.ctrl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == 0u) {
        st_coherent(&P.ctrl->stuck_worker, w.worker);
        st_coherent(&P.ctrl->stuck_pos, w.wb + w.h);
        st_coherent(&P.ctrl->stuck_cnt, ld_coherent(P.cnt + w.wb + w.h));
        st_coherent(&P.ctrl->stuck_h, w.h);
        st_coherent(&P.ctrl->stuck_wcnt, w.wcnt);
      }
    }
    return false;
  }
  return true;
}

// Returns the position of the worker's next ready task, or kExit when its
// list is finished or the launch is being aborted.  Run by one whole wave.
__device__ uint32_t next_task(const ExecParams& P, WorkerState& w, uint32_t lane) {
  for (;;) {
    if (w.pend) {
      const uint32_t b = (uint32_t)__builtin_ctzll(w.pend);
      w.pend &= w.pend - 1;
      w.done |= 1ull << b;
      w.spins = 0;
      w.last = __builtin_amdgcn_s_memrealtime();
      publish_progress(P, w, w.last, lane == 0);
      return w.wb + w.h + b;
    }
    // slide the window past the finished prefix
    const uint32_t adv = (~w.done == 0ull) ? 64u : (uint32_t)__builtin_ctzll(~w.done);
    w.h += adv;
    w.done = adv >= 64u ? 0ull : (w.done >> adv);
    if (adv) w.rescan = true;
    if (w.h >= w.wcnt) return kExit;
    if (P.notify && !w.rescan) {
      // wait for a message: one word per poll instead of the whole window
      const uint32_t b = uni(ld_coherent(P.bell + w.worker * kBellStride));
      if (b == w.seen) {
        if (!idle_step(P, w, lane)) return kExit;
        continue;
      }
      w.seen = b;
    }
    w.pend = ready_scan(lane, P, w);
    if (P.wstamp && lane == 0) {
      uint64_t* ws = P.wstamp + 4 * w.worker;
      const uint64_t now = __builtin_amdgcn_s_memrealtime();
      if (ws[0] == 0) ws[0] = now;
      ws[1] = now;
      ws[2] += 1;
    }
    if (w.pend) {
      w.rescan = true;
      continue;
    }
    w.rescan = false;
    if (P.notify) continue;
    if (!idle_step(P, w, lane)) return kExit;
  }
}

// Residency probe: every worker checks in and then waits (for at most the
// watchdog interval) until all nworkers have checked in.  A worker that saw
// all of them counts itself as resident; the host accepts the worker count
// only if every worker did.  The same kernel (same resources) as the
// executor is used, so the answer holds for the real launch.
__device__ void residency_probe(const ExecParams& P, bool lead) {
  if (lead) __hip_atomic_fetch_add(&P.ctrl->started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    const uint32_t n = uni(ld_coherent(&P.ctrl->started));
    if (n >= P.nworkers) {
      if (lead) __hip_atomic_fetch_add(&P.ctrl->resident, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (__builtin_amdgcn_s_memrealtime() - t0 > P.watchdog_ticks) return;
    __builtin_amdgcn_s_sleep(8);
  }
}

__device__ __forceinline__ void worker_init(WorkerState& w, const ExecParams& P, uint32_t worker) {
  w.worker = worker;
  w.wb = as_const(P.wbase)[worker];
  w.wcnt = as_const(P.wbase)[worker + 1] - w.wb;
  w.h = 0;
  w.done = 0;
  w.pend = 0;
  w.seen = 0;
  w.spins = 0;
  w.last = __builtin_amdgcn_s_memrealtime();
  w.pub = 0;
  w.rescan = true;
  w.pf_pos = kExit;
  w.pf_v = 0;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_exec_wave(ExecParams P) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t worker = uni((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (worker >= P.nworkers || gate_closed(P)) return;
  const WaveTeam tm{lane};
  if (P.diag && lane == 0) __hip_atomic_fetch_add(&P.ctrl->started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  WorkerState w;
  worker_init(w, P, worker);
  for (;;) {
    const uint32_t pos = next_task(P, w, lane);
    if (pos == kExit) break;
    const uint32_t v = pos == w.pf_pos ? w.pf_v : rec_dword(P, pos, lane);
    Rec r;
    run_task(tm, P, pos, v, r);
    complete_edges(tm, P, r);
    if (P.tstamp && lane == 0) P.tstamp[2 * pos + 1] = __builtin_amdgcn_s_memrealtime();
  }
  if (P.wprog && lane == 0) P.wprog[worker] = w.h;
}

// One workgroup per task: wave 0 runs the scheduling state machine and
// stages the chosen position and its record in LDS; every wave then executes
// the same sequence of barriers for each task.
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_exec_block(ExecParams P) {
  __shared__ uint32_t lds[32];
  __shared__ uint32_t cmd;
  __shared__ uint32_t recl[32];
  const uint32_t worker = blockIdx.x;
  if (worker >= P.nworkers || gate_closed(P)) return;
  const BlockTeam tm{threadIdx.x, blockDim.x, lds};
  const uint32_t lane = threadIdx.x & 63u;
  if (P.diag && threadIdx.x == 0)
    __hip_atomic_fetch_add(&P.ctrl->started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  WorkerState w;
  worker_init(w, P, worker);
  for (;;) {
    if (threadIdx.x < 64) {
      const uint32_t pos = next_task(P, w, lane);
      if (pos != kExit) {
        const uint32_t v = pos == w.pf_pos ? w.pf_v : rec_dword(P, pos, lane);
        if (lane < 32) recl[lane] = v;
      }
      if (lane == 0) cmd = pos;
    }
    __syncthreads();
    const uint32_t pos = uni(cmd);
    const uint32_t v = recl[lane & 31u];
    __syncthreads();
    if (pos == kExit) break;
    Rec r;
    run_task(tm, P, pos, v, r);
    complete_edges(tm, P, r);
    if (P.tstamp && threadIdx.x == 0) P.tstamp[2 * pos + 1] = __builtin_amdgcn_s_memrealtime();
    __syncthreads();
  }
  if (P.wprog && threadIdx.x == 0) P.wprog[worker] = w.h;
}

// A gang of P.gang workgroups per task (on different CUs), without a leader:
// every member runs the scheduling loop over the gang's list itself, executes
// its share of each task's work items, adds its digest part to the task's
// digest (zeroed by the reset) and signals every out-edge after draining its
// stores.  A task's counter starts at its in-degree times the gang size, so it
// becomes ready once every member of every predecessor's gang has finished
// its share.  No member waits for another: the members of one gang may run
// different tasks of the list at the same time (each takes its ready entries
// in its own order), and none of the mailbox round trips a leader would need
// (publish the task, collect the arrivals) sits between two dependent tasks.
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_exec_gang(ExecParams P) {
  __shared__ uint32_t lds[32];
  __shared__ uint32_t cmd;
  __shared__ uint32_t recl[32];
  const uint32_t G = P.gang;
  const uint32_t gang = blockIdx.x / G, member = blockIdx.x % G;
  if (gang >= P.nworkers || gate_closed(P)) return;
  GangTeam tm;
  tm.t = threadIdx.x;
  tm.n = blockDim.x;
  tm.lds = lds;
  tm.m = member;
  tm.G = G;
  const uint32_t lane = threadIdx.x & 63u;
  WorkerState w;
  worker_init(w, P, gang);
  for (;;) {
    if (threadIdx.x < 64) {
      const uint32_t pos = next_task(P, w, lane);
      if (pos != kExit) {
        const uint32_t v = pos == w.pf_pos ? w.pf_v : rec_dword(P, pos, lane);
        if (lane < 32) recl[lane] = v;
      }
      if (lane == 0) cmd = pos;
    }
    __syncthreads();
    const uint32_t pos = uni(cmd);
    const uint32_t v = recl[lane & 31u];
    __syncthreads();
    if (pos == kExit) break;
    Rec r;
    const uint32_t d = run_body(tm, P, pos, v, r);
    if (threadIdx.x == 0) __hip_atomic_fetch_add(r.digest + r.tid, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    complete_edges(tm, P, r);
    // diagnostics: a task ends when its last member finishes
    if (P.tstamp && threadIdx.x == 0)
      __hip_atomic_fetch_max(P.tstamp + 2 * pos + 1, __builtin_amdgcn_s_memrealtime(), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }
  if (member == 0 && P.wprog && threadIdx.x == 0) P.wprog[gang] = w.h;
}

// ------------------------------------------------------ ready-queue dispatch
//
// The second dispatch of the executor (Algorithm 1's EXECUTE_OP on the
// vertex a COMPLETED_EDGE made ready), without per-worker lists.  The
// decrement that empties a counter (old value 1) makes its task ready.  A
// worker keeps the first task its own completion made ready as its next task
// (a chain causes no queue traffic) and pushes the others into one ticket
// queue shard (shards taken in turn): one ballot of the ready lanes, one
// atomic add on the shard's tail for all of them, each lane's slot from the
// count of ready lanes below it.  A worker that needs work claims a tile of
// consecutive tickets of its own shard with one atomic add on the head --
// a claim never fails and never retries -- and waits on each claimed slot in
// turn until a pusher has written it; waiting workers poll distinct slots,
// so no address is shared by the waiters.
//
// Termination needs no per-task counter: every task precedes some sink (a
// task without out-edges), so the launch is over once every sink has run.
// Workers count the sinks they finished and add the count to one word only
// when they find their next slot empty; the addition that completes the sink
// total pushes qsent exit sentinels into every shard.  A worker claims a new
// tile only after consuming its previous one, so at most one tile per worker
// (plus one straddling the last task ticket) reaches past the task tickets
// of a shard: qsent = tile x (workers of the shard + 1) sentinels fill every
// ticket ever claimed.  No worker waits for a particular other worker, so
// this dispatch needs no co-residency.

struct QueueState {
  uint32_t worker, shard, pshard;  // claims from `shard`; next push into `pshard`
  uint32_t local;                  // ready task kept by this worker (kExit: none)
  uint32_t tile_h, tile_n, tile_i; // claimed tickets [tile_h, tile_h + tile_n), next tile_i
  uint32_t sinks;                  // sinks finished since the last report
  uint64_t pub;                    // time this worker last published Ctrl::progress
};

__device__ __forceinline__ uint32_t* q_head(const ExecParams& P, uint32_t s) { return P.qctl + s * kQLine; }
__device__ __forceinline__ uint32_t* q_tail(const ExecParams& P, uint32_t s) {
  return P.qctl + (P.qshards + s) * kQLine;
}
__device__ __forceinline__ uint32_t* q_sinks(const ExecParams& P) { return P.qctl + 2u * P.qshards * kQLine; }

// Workgroups are dealt to the 8 XCDs round-robin by workgroup index.
__device__ __forceinline__ void queue_init(QueueState& q, const ExecParams& P, uint32_t worker) {
  q.worker = worker;
  q.shard = blockIdx.x & 7u & (P.qshards - 1u);
  q.pshard = q.shard;
  q.local = kExit;
  q.tile_h = q.tile_n = q.tile_i = 0;
  q.sinks = 0;
  q.pub = 0;
}

// Raises the abort flag; the first abort records where it happened.
__device__ void queue_abort(const ExecParams& P, const QueueState& q, uint32_t lane, uint32_t ticket) {
  if (lane != 0) return;
  const uint32_t prev = __hip_atomic_fetch_add(&P.ctrl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (prev == 0u) {
    st_coherent(&P.ctrl->stuck_worker, q.worker);
    st_coherent(&P.ctrl->stuck_pos, ticket);
    st_coherent(&P.ctrl->stuck_cnt, ld_coherent(q_sinks(P)));
    st_coherent(&P.ctrl->stuck_h, q.shard);
    st_coherent(&P.ctrl->stuck_wcnt, P.npos);
  }
}

// The end of the launch: qsent exit sentinels into every shard.
__device__ void queue_finish(const ExecParams& P, uint32_t lane) {
  for (uint32_t s = 0; s < P.qshards; ++s) {
    uint32_t base = 0;
    if (lane == 0) base = __hip_atomic_fetch_add(q_tail(P, s), P.qsent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    base = rl(base, 0);
    uint32_t* slot = P.q + (size_t)s * P.qcap;
    for (uint32_t i = lane; i < P.qsent; i += 64u)
      if (base + i < P.qcap) st_coherent(slot + base + i, kQExit);
  }
}

// Reports the sinks this worker finished; the report that completes the
// total ends the launch.
__device__ __forceinline__ void queue_report(const ExecParams& P, QueueState& q, uint32_t lane) {
  if (q.sinks == 0u) return;
  uint32_t old = 0;
  if (lane == 0) old = __hip_atomic_fetch_add(q_sinks(P), q.sinks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  old = rl(old, 0);
  const bool last = old + q.sinks == P.nsinks;
  q.sinks = 0;
  if (last) queue_finish(P, lane);
}

__device__ __forceinline__ void queue_progress(const ExecParams& P, QueueState& q, uint32_t lane) {
  const uint64_t now = __builtin_amdgcn_s_memrealtime();
  if (now - q.pub < P.progress_ticks) return;
  q.pub = now;
  if (lane == 0) __hip_atomic_fetch_max(&P.ctrl->progress, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Position of the worker's next task, or kExit at the end of the launch (or
// when it is being aborted).  Run by one whole wave.
__device__ uint32_t queue_next(const ExecParams& P, QueueState& q, uint32_t lane) {
  if (q.local != kExit) {
    const uint32_t pos = q.local;
    q.local = kExit;
    queue_progress(P, q, lane);
    return pos;
  }
  if (q.tile_i == q.tile_n) {
    uint32_t h = 0;
    if (lane == 0) h = __hip_atomic_fetch_add(q_head(P, q.shard), P.qtile, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    q.tile_h = rl(h, 0);
    q.tile_n = P.qtile;
    q.tile_i = 0;
  }
  const uint32_t t = q.tile_h + q.tile_i;
  if (t >= P.qcap) {  // beyond every sentinel: the protocol's bound was broken
    queue_abort(P, q, lane, t);
    return kExit;
  }
  const uint32_t* slot = P.q + (size_t)q.shard * P.qcap + t;
  uint32_t v = uni(ld_coherent(slot));
  if (v == kQEmpty) {
    queue_report(P, q, lane);  // nothing to run now: report the finished sinks first
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    // a fixed back-off here, not the growing one of the lists: a queue
    // worker waits for whichever task is pushed next, and in the serving
    // loop a late claim delays a request (median latency 9.7 ms with the
    // fixed back-off, 11.4 ms with the growing one, same box)
    for (uint32_t spins = 1;; ++spins) {
      const uint32_t nap = spins < 64 ? 1u : P.idle_sleep;
      for (uint32_t i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(2);
      v = uni(ld_coherent(slot));
      if (v != kQEmpty) break;
      if ((spins & 63u) == 0u) {
        if (uni(ld_coherent(&P.ctrl->abort)) != 0u) return kExit;
        if (stalled(P, t0, __builtin_amdgcn_s_memrealtime()) || (P.spin_limit != 0u && spins >= P.spin_limit)) {
          queue_abort(P, q, lane, t);
          return kExit;
        }
      }
    }
  }
  ++q.tile_i;
  if (v == kQExit) return kExit;
  queue_progress(P, q, lane);
  return v;
}

// One wave's part of a completion: `ready` marks the lanes whose decrement
// emptied the counter of `dst`.  The scheduling wave (keep) holds on to the
// first of them when it has no next task yet; the rest are pushed into the
// next shard in turn with one atomic on its tail.
__device__ __forceinline__ void queue_push(const ExecParams& P, QueueState& q, bool keep, uint32_t lane, bool ready,
                                           uint32_t dst) {
  uint64_t m = uni64(__ballot(ready));
  if (!m) return;
  if (keep && q.local == kExit) {
    const uint32_t first = (uint32_t)__builtin_ctzll(m);
    q.local = __builtin_amdgcn_readlane(dst, first);
    m &= m - 1;
    if (lane == first) ready = false;
    if (!m) return;
  }
  const uint32_t s = q.pshard;
  q.pshard = (q.pshard + 1u) & (P.qshards - 1u);
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  uint32_t base = 0;
  if (lane == leader)
    base = __hip_atomic_fetch_add(q_tail(P, s), (uint32_t)__builtin_popcountll(m), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = __builtin_amdgcn_readlane(base, leader);
  if (ready) {
    const uint32_t idx = base + (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1ull));
    if (idx < P.qcap) st_coherent(P.q + (size_t)s * P.qcap + idx, dst);
  }
  // a shard holds at most every task once plus the sentinels, so a full
  // shard means a broken protocol: stop the launch rather than lose a task
  if (base + (uint32_t)__builtin_popcountll(m) > P.qcap) queue_abort(P, q, lane, base);
}

// COMPLETED_EDGE for every out-edge, then the pushes (one per wave with
// ready successors).  The payload stores are drained first, as in the list
// dispatch.
template <class Team>
__device__ __forceinline__ void complete_edges_q(const Team& tm, const ExecParams& P, const Rec& r, QueueState& q,
                                                 bool keep) {
  vm_drain();
  tm.sync();
  const uint32_t lane = tm.t & 63u;
  for (uint32_t j0 = 0; j0 < r.nsucc; j0 += tm.size()) {
    const uint32_t j = j0 + tm.t;
    bool ready = false;
    uint32_t dst = 0;
    if (j < r.nsucc) {
      dst = j0 == 0 ? r.succ0 : P.succ_pos[r.succ_beg + j];
      ready = __hip_atomic_fetch_sub(P.cnt + dst, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1u;
    }
    queue_push(P, q, keep, lane, ready, dst);
  }
}

// Per-graph completion (launches that report graphs as they finish): a
// finished sink adds one to its graph's count; the addition that completes
// it stores the launch's sequence number into the graph's flag in host
// memory.  Every task of the graph precedes one of its sinks, and every
// sink's stores were drained before its addition, so the graph's results are
// in memory when the flag is seen.
__device__ __forceinline__ void graph_sink_done(const ExecParams& P, uint32_t graph, bool lead) {
  if (!P.gdone || !lead) return;
  const uint32_t old = __hip_atomic_fetch_add(P.gdone + graph, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (old + 1u == as_const(P.gtab)[graph].nsinks)
    __hip_atomic_store(P.gflag + graph, P.gseq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_exec_wave_q(ExecParams P) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t worker = uni((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (worker >= P.nworkers || gate_closed(P)) return;
  const WaveTeam tm{lane};
  if (P.diag && lane == 0) __hip_atomic_fetch_add(&P.ctrl->started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  QueueState q;
  queue_init(q, P, worker);
  for (;;) {
    const uint32_t pos = queue_next(P, q, lane);
    if (pos == kExit) break;
    Rec r;
    run_task(tm, P, pos, rec_dword(P, pos, lane), r);
    if (r.nsucc == 0u) ++q.sinks;
    complete_edges_q(tm, P, r, q, true);
    if (r.nsucc == 0u) graph_sink_done(P, r.graph, lane == 0);
    if (P.tstamp && lane == 0) P.tstamp[2 * pos + 1] = __builtin_amdgcn_s_memrealtime();
  }
}

// One workgroup per task: wave 0 takes the tasks and stages the record in
// LDS; every wave pushes the successors its lanes made ready.
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_exec_block_q(ExecParams P) {
  __shared__ uint32_t lds[32];
  __shared__ uint32_t cmd;
  __shared__ uint32_t recl[32];
  const uint32_t worker = blockIdx.x;
  if (worker >= P.nworkers || gate_closed(P)) return;
  const BlockTeam tm{threadIdx.x, blockDim.x, lds};
  const uint32_t lane = threadIdx.x & 63u;
  if (P.diag && threadIdx.x == 0)
    __hip_atomic_fetch_add(&P.ctrl->started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  QueueState q;
  queue_init(q, P, worker);
  for (;;) {
    if (threadIdx.x < 64) {
      const uint32_t pos = queue_next(P, q, lane);
      if (pos != kExit && lane < 32) recl[lane] = rec_dword(P, pos, lane);
      if (lane == 0) cmd = pos;
    }
    __syncthreads();
    const uint32_t pos = uni(cmd);
    const uint32_t v = recl[lane & 31u];
    __syncthreads();
    if (pos == kExit) break;
    Rec r;
    run_task(tm, P, pos, v, r);
    if (threadIdx.x < 64 && r.nsucc == 0u) ++q.sinks;
    complete_edges_q(tm, P, r, q, threadIdx.x < 64);
    if (r.nsucc == 0u) graph_sink_done(P, r.graph, threadIdx.x == 0);
    if (P.tstamp && threadIdx.x == 0) P.tstamp[2 * pos + 1] = __builtin_amdgcn_s_memrealtime();
    __syncthreads();
  }
}

// Empties the slots the previous launch filled: [0, tail) of every shard
// (the tails are still the previous launch's; k_queue_seed resets them).
__global__ __launch_bounds__(256) void k_queue_clear(ExecParams P) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t s = 0; s < P.qshards; ++s) {
    uint32_t t = *q_tail(P, s);
    if (t > P.qcap) t = P.qcap;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < t; i += stride) P.q[(size_t)s * P.qcap + i] = kQEmpty;
  }
}

// Sources dealt round-robin over the shards; heads, tails and the sink count
// reset.
__global__ __launch_bounds__(256) void k_queue_seed(ExecParams P) {
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t i = gid; i < P.nsrc; i += stride) P.q[(size_t)(i % P.qshards) * P.qcap + i / P.qshards] = P.qsrc[i];
  if (gid < P.qshards) {
    *q_head(P, gid) = 0u;
    *q_tail(P, gid) = (P.nsrc + P.qshards - 1u - gid) / P.qshards;
  }
  if (gid == 0) *q_sinks(P) = 0u;
}

// Residency probes: the executors' launch bounds and occupancy attributes
// (so the same number of blocks fits per CU), kept as kernels of their own so
// that kernel traces of real launches are not mixed with probe launches.
// Every wave of a block stays until the probe is over, so a probe block
// occupies what an executor block occupies.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_probe_wave(ExecParams P) {
  const uint32_t worker = uni((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (worker >= P.nworkers) return;
  residency_probe(P, (threadIdx.x & 63u) == 0);
}

__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_probe_block(ExecParams P) {
  if (blockIdx.x >= P.nworkers) return;
  if (threadIdx.x < 64) residency_probe(P, threadIdx.x == 0);
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_reset(ExecParams P) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P.npos; i += stride) {
    P.cnt[i] = P.indeg[i];
    if (P.execs) P.execs[i] = 0;
  }
  // gangs add their members' digest parts into the digest words
  if (P.gang > 1)
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P.npos; i += stride) {
      const uint32_t* rd = reinterpret_cast<const uint32_t*>(P.rec + i);
      P.gtab[rd[kDwGraph]].digest[rd[kDwTid]] = 0;
    }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P.nworkers; i += stride) {
    P.bell[i * kBellStride] = 0;
    if (P.wprog) P.wprog[i] = 0xFFFFFFFFu;
    if (P.wstamp)
      for (int k = 0; k < 4; ++k) P.wstamp[4 * i + k] = 0;
  }
  if (P.tstamp)
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * P.npos; i += stride) P.tstamp[i] = 0;
  // an abort of an earlier, not yet inspected launch stays visible
  if (blockIdx.x == 0 && threadIdx.x == 0) P.ctrl->sticky += P.ctrl->abort;
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < 8) (&P.ctrl->abort)[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P.ctrl->progress = 0;
    P.ctrl->precond = 0;
  }
}

// Comparator: one launch runs one task; ordering comes from the stream or
// from the hipGraph's dependency edges, so no counter is touched.
__global__ __launch_bounds__(64) void k_one_task(ExecParams P, uint32_t pos) {
  const WaveTeam tm{threadIdx.x};
  Rec r;
  run_task(tm, P, pos, rec_dword(P, pos, threadIdx.x), r);
}

// -------------------------------------------- records built on the device

// Last graph whose `field` is <= x (the table ascends in it; graphs without
// tasks share their successor's base, so the last such graph is the one that
// holds x).
template <uint32_t GraphSrc::*F>
__device__ __forceinline__ uint32_t graph_of(const GraphSrc* g, uint32_t ng, uint32_t x) {
  uint32_t lo = 0, hi = ng;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (g[mid].*F <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One thread per position: the record of the task at that position (layout
// order = graph order, task ids ascending), its slices of the predecessor
// address and successor position arrays, and its counter reset value; then
// one thread per source: the launch's source list.
__global__ __launch_bounds__(256) void k_build_records(const GraphSrc* gsrc, uint32_t ng, uint32_t npos, uint32_t nsrc,
                                                       TaskRec* rec, uint64_t* pred_addr, uint32_t* succ_pos,
                                                       uint32_t* indeg, uint32_t* src) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npos; p += stride) {
    const uint32_t gi = graph_of<&GraphSrc::pos_base>(gsrc, ng, p);
    const GraphSrc& g = gsrc[gi];
    const uint32_t v = p - g.pos_base;
    TaskRec r;
    memset(&r, 0, sizeof(r));
    r.tid = v;
    r.graph = gi;
    r.rounds = g.rounds[v];
    const uint64_t wbytes = (uint64_t)g.n * 4u;
    // the inline lists are filled with constant indices so that the record
    // stays in registers (a variable index would put it in scratch memory)
    if (g.mode == 1) {
      r.out = g.payload + (uint64_t)(g.slot ? g.slot[v] : v) * wbytes;
      const uint32_t d0 = g.pred_ptr[v], d1 = g.pred_ptr[v + 1];
      r.npred = d1 - d0;
      r.pred_beg = g.pred_base + d0;
#pragma unroll
      for (uint32_t k = 0; k < kInPred; ++k)
        if (k < r.npred) {
          const uint32_t q = g.preds[d0 + k];
          r.pred[k] = g.payload + (uint64_t)(g.slot ? g.slot[q] : q) * wbytes;
        }
      for (uint32_t j = d0; j < d1; ++j) {
        const uint32_t q = g.preds[j];
        pred_addr[g.pred_base + j] = g.payload + (uint64_t)(g.slot ? g.slot[q] : q) * wbytes;
      }
    } else {
      const uint32_t a0 = g.req_ptr[v];
      r.out = (uint64_t)(g.reqs + a0);
      r.nreq = g.req_ptr[v + 1] - a0;
    }
    const uint32_t s0 = g.succ_ptr[v], s1 = g.succ_ptr[v + 1];
    r.nsucc = s1 - s0;
    r.succ_beg = g.succ_base + s0;
#pragma unroll
    for (uint32_t k = 0; k < kInSucc; ++k)
      if (k < r.nsucc) r.succ[k] = g.pos_base + g.succ[s0 + k];
    for (uint32_t j = s0; j < s1; ++j) succ_pos[g.succ_base + j] = g.pos_base + g.succ[j];
    rec[p] = r;
    indeg[p] = g.indeg[v];
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nsrc; i += stride) {
    const GraphSrc& g = gsrc[graph_of<&GraphSrc::src_base>(gsrc, ng, i)];
    src[i] = g.pos_base + g.src[i - g.src_base];
  }
}

// Pre-condition vertices met by the host or by another launch (Section 4.1):
// lane i polls flag i (system-scope loads of pinned host memory) until every
// flag holds at least its value, or gives up after timeout_ticks.
__global__ __launch_bounds__(64) void k_wait_flags(FlagWait fw, Ctrl* ctrl, uint64_t timeout_ticks) {
  const uint32_t lane = threadIdx.x;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    bool met = true;
    if (lane < fw.n) met = __hip_atomic_load(fw.addr[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) >= fw.value[lane];
    const uint64_t unmet = __ballot(!met);
    if (unmet == 0ull) return;
    if (__builtin_amdgcn_s_memrealtime() - t0 > timeout_ticks) {
      if (lane == 0) {
        st_coherent(&ctrl->precond, 1u + (uint32_t)__builtin_ctzll(unmet));
        __hip_atomic_fetch_add(&ctrl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return;
    }
    __builtin_amdgcn_s_sleep(32);
  }
}

// Post-condition vertex: runs after the launch in stream order, so every
// task of it has finished; publishes them (system-scope release) and sets the
// flag, unless the launch was abandoned.
__global__ __launch_bounds__(64) void k_set_flag(uint32_t* flag, uint32_t value, const Ctrl* ctrl) {
  if (threadIdx.x != 0) return;
  if (__hip_atomic_load(&ctrl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
  __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(256) void k_fill(uint32_t* p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_build_records(const GraphSrc* gsrc, uint32_t ng, uint32_t npos, uint32_t nsrc, TaskRec* rec,
                                uint64_t* pred_addr, uint32_t* succ_pos, uint32_t* indeg, uint32_t* src,
                                hipStream_t s) {
  const uint32_t n = npos > nsrc ? npos : nsrc;
  uint32_t blocks = (n + 255u) / 256u;
  if (blocks > 8192u) blocks = 8192u;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_build_records, dim3(blocks), dim3(256), 0, s, gsrc, ng, npos, nsrc, rec, pred_addr, succ_pos,
                     indeg, src);
  return hipGetLastError();
}

hipError_t launch_fill(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill, dim3((uint32_t)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}


hipError_t launch_wait_flags(const FlagWait& fw, Ctrl* ctrl, uint64_t timeout_ticks, hipStream_t s) {
  if (fw.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_wait_flags, dim3(1), dim3(64), 0, s, fw, ctrl, timeout_ticks);
  return hipGetLastError();
}

hipError_t launch_set_flag(uint32_t* flag, uint32_t value, const Ctrl* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, s, flag, value, ctrl);
  return hipGetLastError();
}

hipError_t launch_reset(const ExecParams& p, hipStream_t s) {
  uint32_t blocks = (p.npos + 255u) / 256u;
  if (blocks > 4096u) blocks = 4096u;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_exec(const ExecParams& p, uint32_t mapping, uint32_t wg_waves, uint32_t grid_blocks,
                       hipStream_t s) {
  if (p.residency_probe) {
    if (mapping == 1) hipLaunchKernelGGL(k_probe_wave, dim3(grid_blocks), dim3(256), 0, s, p);
    else hipLaunchKernelGGL(k_probe_block, dim3(grid_blocks), dim3(wg_waves * 64u), 0, s, p);
  } else if (mapping == 1) {
    hipLaunchKernelGGL(k_exec_wave, dim3(grid_blocks), dim3(256), 0, s, p);
  } else if (mapping == 2) {
    hipLaunchKernelGGL(k_exec_block, dim3(grid_blocks), dim3(wg_waves * 64u), 0, s, p);
  } else {
    hipLaunchKernelGGL(k_exec_gang, dim3(grid_blocks), dim3(wg_waves * 64u), 0, s, p);
  }
  return hipGetLastError();
}

hipError_t launch_queue_clear(const ExecParams& p, hipStream_t s) {
  uint32_t blocks = (p.qcap + 255u) / 256u;
  if (blocks > 4096u) blocks = 4096u;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_queue_clear, dim3(blocks), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_queue_reset(const ExecParams& p, hipStream_t s) {
  uint32_t blocks = (p.npos + 255u) / 256u;
  if (blocks > 4096u) blocks = 4096u;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_queue_clear, dim3(blocks), dim3(256), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint32_t sb = (p.nsrc + 255u) / 256u;
  if (sb > 4096u) sb = 4096u;
  if (sb == 0) sb = 1;
  hipLaunchKernelGGL(k_queue_seed, dim3(sb), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_exec_queue(const ExecParams& p, uint32_t mapping, uint32_t wg_waves, uint32_t grid_blocks,
                             hipStream_t s) {
  if (mapping == 1) hipLaunchKernelGGL(k_exec_wave_q, dim3(grid_blocks), dim3(256), 0, s, p);
  else hipLaunchKernelGGL(k_exec_block_q, dim3(grid_blocks), dim3(wg_waves * 64u), 0, s, p);
  return hipGetLastError();
}

int exec_blocks_per_cu(uint32_t mapping, uint32_t wg_waves) {
  int nb = 0;
  hipError_t e;
  if (mapping == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_exec_wave, 256, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_exec_block, (int)(wg_waves * 64u), 0);
  if (e != hipSuccess) return -1;
  return nb;
}

hipError_t launch_one_task(const ExecParams& p, uint32_t pos, hipStream_t s) {
  hipLaunchKernelGGL(k_one_task, dim3(1), dim3(64), 0, s, p, pos);
  return hipGetLastError();
}

const void* one_task_kernel() { return (const void*)k_one_task; }

}  // namespace tg
