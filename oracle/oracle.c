/*
 * Reference oracle for the task-DAG executor.  TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential C.  Nothing here is used by the product path; only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * load this library.  It shares no source, header or helper with the HIP
 * library: every definition below is written out from the paper and from the
 * published definitions it relies on.
 *
 * What the method computes ("Yadav et al., On the Duality of Task and Actor
 * Programming Models"):
 *   - Explicit mode (Figure 3, Section 4.2 and Algorithm 1): a task runs once,
 *     after every task whose completion event it was predicated on.  Because
 *     topologically unordered vertices may run in any order (Section 4.2), the
 *     result is the one any topological order gives; the oracle uses Kahn's
 *     algorithm with a FIFO queue and ascending-id tie break.
 *   - Implicit mode (Section 2, implicitly-parallel systems; Section 5): tasks
 *     declare the data they read and write, the runtime infers dependences, and
 *     the result equals running the tasks sequentially in program order.
 *
 * Readings where the paper is silent (the paper uses a floating-point busy
 * loop as task body, Section 6.1; here the body is an exact integer mix):
 *   - mix_round(x) = M(xorshift32(x)), xorshift32 = Marsaglia's (13,17,5)
 *     triple, M(y) = y*0x9E3779B1 + 0x7F4A7C15 mod 2^32; mix_R = R rounds.
 *   - sm64 = SplitMix64 output function (Steele, Lea, Flood 2014);
 *     h32(seed,stream,idx) = low32(sm64(sm64(seed ^ (stream<<32)) ^ idx)).
 *   - Source task payload word k: h32(seed, 1, (id<<16)|k).
 *   - Non-source input word k: wrap sum over the SET of distinct predecessors.
 *   - out[k] = mix_R(in[k] ^ id); digest d = sum_k out[k]*(2k+1) mod 2^32;
 *     checksum = sum_v (u64)d(v)*(2v+1) mod 2^64.
 *   - Conflict rule (implicit): tasks j<k conflict iff an interval of j and an
 *     interval of k overlap and at least one of the two is read-write; every
 *     conflicting pair is an edge j->k (no transitive reduction, Section 5).
 *   - Implicit body of task k: c = wrap sum of the current values of its
 *     read-only elements; each read-write element e, in declaration order,
 *     becomes mix_R(A[e] ^ c ^ k); the digest enumerates the written elements
 *     in declaration order with weights 2j+1.  Initial A[e] = h32(seed, 2, e).
 *
 * Parity pins (tests/test_oracle_*.py): published SplitMix64 outputs,
 * Marsaglia's published xorshift32 example, an independent inverse of the mix,
 * exactly-once / precedence checks, every-topological-order invariance on
 * small graphs (including the Figure 6 DAG), local re-derivation of every
 * payload from its predecessors, brute-force element-set conflict checks and
 * a closed-form edge count for the implicit workload, and program order vs
 * DAG order for implicit execution.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ECYCLE (-3)
#define OR_EORDER (-4)

/* ---------------------------------------------------------------- hashing */

/* SplitMix64 output for counter z (add the golden gamma, then the two
 * xor-shift-multiply finalisation steps). */
uint64_t or_sm64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint32_t or_h32(uint64_t seed, uint32_t stream, uint64_t idx) {
  uint64_t key = or_sm64(seed ^ ((uint64_t)stream << 32));
  return (uint32_t)(or_sm64(key ^ idx) & 0xFFFFFFFFull);
}

/* Marsaglia's xorshift32 step with the (13, 17, 5) triple. */
uint32_t or_xorshift32(uint32_t x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}

uint32_t or_mix(uint32_t x, uint32_t rounds) {
  uint32_t r;
  for (r = 0; r < rounds; r++) {
    x = or_xorshift32(x);
    x = x * 0x9E3779B1u + 0x7F4A7C15u;
  }
  return x;
}

/* ------------------------------------------------------- explicit graphs */

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

/* Distinct predecessor sets (Figure 3: an operation waits on a SET of events).
 * A predecessor must name an already created task, so p < v. */
typedef struct {
  uint64_t* ptr;  /* N+1 */
  uint32_t* idx;  /* distinct preds, ascending per task */
} or_sets;

static int build_sets(uint32_t N, const uint64_t* pred_ptr, const uint32_t* preds, or_sets* s) {
  uint64_t total = pred_ptr[N], v, j, w;
  s->ptr = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)N + 1));
  s->idx = (uint32_t*)malloc(sizeof(uint32_t) * (total ? total : 1));
  if (!s->ptr || !s->idx) return OR_ENOMEM;
  s->ptr[0] = 0;
  w = 0;
  for (v = 0; v < N; v++) {
    uint64_t b = pred_ptr[v], e = pred_ptr[v + 1], start = w;
    if (e < b) return OR_EINVAL;
    for (j = b; j < e; j++) {
      if (preds[j] >= v) return OR_EINVAL;
      s->idx[w++] = preds[j];
    }
    qsort(s->idx + start, (size_t)(w - start), sizeof(uint32_t), cmp_u32);
    /* drop duplicates */
    {
      uint64_t r, o = start;
      for (r = start; r < w; r++)
        if (r == start || s->idx[r] != s->idx[o - 1]) s->idx[o++] = s->idx[r];
      w = o;
    }
    s->ptr[v + 1] = w;
  }
  return OR_OK;
}

static void free_sets(or_sets* s) {
  free(s->ptr);
  free(s->idx);
}

/* Body of task v (explicit mode): gather, xor id, mix, digest. */
static uint32_t run_task(uint32_t v, uint32_t n, const or_sets* s, const uint32_t* rounds,
                         uint64_t seed, uint32_t* payload) {
  uint32_t k;
  uint32_t d = 0;
  uint64_t b = s->ptr[v], e = s->ptr[v + 1], j;
  for (k = 0; k < n; k++) {
    uint32_t in = 0;
    if (b == e) {
      in = or_h32(seed, 1, ((uint64_t)v << 16) | k);
    } else {
      for (j = b; j < e; j++) in += payload[(size_t)s->idx[j] * n + k];
    }
    payload[(size_t)v * n + k] = or_mix(in ^ v, rounds[v]);
  }
  for (k = 0; k < n; k++) d += payload[(size_t)v * n + k] * (2u * k + 1u);
  return d;
}

static uint64_t checksum_of(uint32_t N, const uint32_t* digest) {
  uint64_t c = 0, v;
  for (v = 0; v < N; v++) c += (uint64_t)digest[v] * (2ull * v + 1ull);
  return c;
}

/*
 * Kahn's algorithm, FIFO queue seeded with the sources in ascending id
 * (Algorithm 1: INIT starts every vertex without in-edges; COMPLETED_EDGE
 * removes one in-edge and starts the vertex once none remain; EXECUTE_OP runs
 * the vertex and then notifies each out-edge).
 *
 * Inputs: pred lists in creation order (duplicates allowed, p < v), per-task
 * rounds, seed.  Outputs: payload (N*n words, may be NULL), digest (N),
 * order (N, may be NULL: the execution order), checksum (may be NULL).
 */
int or_exec_explicit(uint32_t N, uint32_t n, const uint64_t* pred_ptr, const uint32_t* preds,
                     const uint32_t* rounds, uint64_t seed, uint32_t* payload_out,
                     uint32_t* digest, uint32_t* order, uint64_t* checksum) {
  or_sets s;
  uint64_t *succ_ptr = NULL, v, j;
  uint32_t *succ = NULL, *pending = NULL, *queue = NULL, *payload = payload_out, *fill = NULL;
  uint8_t* done = NULL;
  uint64_t qh = 0, qt = 0, processed = 0;
  int rc = OR_OK;
  memset(&s, 0, sizeof(s));
  if (n == 0 || n > 65536) return OR_EINVAL;
  if ((rc = build_sets(N, pred_ptr, preds, &s)) != OR_OK) goto out;
  if (!payload) payload = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N * n + 4);
  succ_ptr = (uint64_t*)calloc((size_t)N + 1, sizeof(uint64_t));
  succ = (uint32_t*)malloc(sizeof(uint32_t) * (s.ptr[N] ? s.ptr[N] : 1));
  pending = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)N + 1));
  queue = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)N + 1));
  fill = (uint32_t*)calloc((size_t)N + 1, sizeof(uint32_t));
  done = (uint8_t*)calloc((size_t)N + 1, 1);
  if (!payload || !succ_ptr || !succ || !pending || !queue || !fill || !done) { rc = OR_ENOMEM; goto out; }
  /* successor lists: out-edges of every vertex */
  for (v = 0; v < N; v++)
    for (j = s.ptr[v]; j < s.ptr[v + 1]; j++) succ_ptr[s.idx[j] + 1]++;
  for (v = 0; v < N; v++) succ_ptr[v + 1] += succ_ptr[v];
  for (v = 0; v < N; v++)
    for (j = s.ptr[v]; j < s.ptr[v + 1]; j++) {
      uint32_t p = s.idx[j];
      succ[succ_ptr[p] + fill[p]++] = (uint32_t)v;
    }
  /* INIT: reset the in-edge counters and start every source */
  for (v = 0; v < N; v++) {
    pending[v] = (uint32_t)(s.ptr[v + 1] - s.ptr[v]);
    if (pending[v] == 0) queue[qt++] = (uint32_t)v;
  }
  while (qh < qt) {
    uint32_t u = queue[qh++];
    if (done[u]) { rc = OR_EORDER; goto out; }
    for (j = s.ptr[u]; j < s.ptr[u + 1]; j++)
      if (!done[s.idx[j]]) { rc = OR_EORDER; goto out; }
    digest[u] = run_task(u, n, &s, rounds, seed, payload);
    done[u] = 1;
    if (order) order[processed] = u;
    processed++;
    /* EXECUTE_OP notifies every out-edge; COMPLETED_EDGE starts at zero */
    for (j = succ_ptr[u]; j < succ_ptr[u + 1]; j++) {
      uint32_t w = succ[j];
      if (--pending[w] == 0) queue[qt++] = w;
    }
  }
  if (processed != N) { rc = OR_ECYCLE; goto out; }
  if (checksum) *checksum = checksum_of(N, digest);
out:
  if (payload != payload_out) free(payload);
  free(succ_ptr); free(succ); free(pending); free(queue); free(fill); free(done);
  free_sets(&s);
  return rc;
}

/*
 * Run the tasks in a caller-given order; the order must be topological
 * (every predecessor earlier, every task exactly once), else OR_EORDER.
 * Used to check that every topological order gives one result.
 */
int or_exec_in_order(uint32_t N, uint32_t n, const uint64_t* pred_ptr, const uint32_t* preds,
                     const uint32_t* rounds, uint64_t seed, const uint32_t* order,
                     uint32_t* payload_out, uint32_t* digest, uint64_t* checksum) {
  or_sets s;
  uint32_t* payload = payload_out;
  uint8_t* done = NULL;
  uint64_t i, j;
  int rc = OR_OK;
  memset(&s, 0, sizeof(s));
  if (n == 0 || n > 65536) return OR_EINVAL;
  if ((rc = build_sets(N, pred_ptr, preds, &s)) != OR_OK) goto out;
  if (!payload) payload = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N * n + 4);
  done = (uint8_t*)calloc((size_t)N + 1, 1);
  if (!payload || !done) { rc = OR_ENOMEM; goto out; }
  for (i = 0; i < N; i++) {
    uint32_t u = order[i];
    if (u >= N || done[u]) { rc = OR_EORDER; goto out; }
    for (j = s.ptr[u]; j < s.ptr[u + 1]; j++)
      if (!done[s.idx[j]]) { rc = OR_EORDER; goto out; }
    digest[u] = run_task(u, n, &s, rounds, seed, payload);
    done[u] = 1;
  }
  if (checksum) *checksum = checksum_of(N, digest);
out:
  if (payload != payload_out) free(payload);
  free(done);
  free_sets(&s);
  return rc;
}

/* -------------------------------------------------------- implicit graphs */

/* Region requirement list in program order: task k owns requirements
 * req_ptr[k] .. req_ptr[k+1]-1, each a half-open interval [lo, hi) of the
 * index space with privilege priv (1 = read-only, 2 = read-write). */
#define OR_RO 1u
#define OR_RW 2u

/* Two half-open intervals share an element iff max(lo) < min(hi); an empty
 * interval shares nothing. */
static int overlap(uint64_t lo1, uint64_t hi1, uint64_t lo2, uint64_t hi2) {
  uint64_t lo = lo1 > lo2 ? lo1 : lo2, hi = hi1 < hi2 ? hi1 : hi2;
  return lo < hi;
}

static int check_reqs(uint32_t N, const uint64_t* req_ptr, const uint64_t* lo, const uint64_t* hi,
                      const uint32_t* priv, uint64_t space) {
  uint64_t k, a, b;
  for (k = 0; k < N; k++) {
    if (req_ptr[k + 1] < req_ptr[k]) return OR_EINVAL;
    for (a = req_ptr[k]; a < req_ptr[k + 1]; a++) {
      if (lo[a] > hi[a] || hi[a] > space) return OR_EINVAL;
      if (priv[a] != OR_RO && priv[a] != OR_RW) return OR_EINVAL;
      /* within one task, a read-write interval overlaps no other interval */
      for (b = req_ptr[k]; b < req_ptr[k + 1]; b++) {
        if (a == b) continue;
        if ((priv[a] == OR_RW || priv[b] == OR_RW) && overlap(lo[a], hi[a], lo[b], hi[b])) return OR_EINVAL;
      }
    }
  }
  return OR_OK;
}

/* Body of implicit task k on the array A (see the header comment). */
static uint32_t run_implicit_task(uint32_t k, const uint64_t* req_ptr, const uint64_t* lo,
                                  const uint64_t* hi, const uint32_t* priv, uint32_t rounds,
                                  uint32_t* A) {
  uint64_t a, e;
  uint32_t c = 0, d = 0, j = 0;
  for (a = req_ptr[k]; a < req_ptr[k + 1]; a++)
    if (priv[a] == OR_RO)
      for (e = lo[a]; e < hi[a]; e++) c += A[e];
  for (a = req_ptr[k]; a < req_ptr[k + 1]; a++)
    if (priv[a] == OR_RW)
      for (e = lo[a]; e < hi[a]; e++) {
        A[e] = or_mix(A[e] ^ c ^ k, rounds);
        d += A[e] * (2u * j + 1u);
        j++;
      }
  return d;
}

static void init_array(uint32_t* A, uint64_t space, uint64_t seed) {
  uint64_t e;
  for (e = 0; e < space; e++) A[e] = or_h32(seed, 2, e);
}

/* Sequential program order: the semantics an implicitly parallel system
 * promises (Section 5).  A (space words) is written with the final array. */
int or_implicit_program_order(uint32_t N, const uint64_t* req_ptr, const uint64_t* lo,
                              const uint64_t* hi, const uint32_t* priv, const uint32_t* rounds,
                              uint64_t seed, uint64_t space, uint32_t* A, uint32_t* digest,
                              uint64_t* checksum) {
  uint32_t k;
  int rc = check_reqs(N, req_ptr, lo, hi, priv, space);
  if (rc != OR_OK) return rc;
  init_array(A, space, seed);
  for (k = 0; k < N; k++) digest[k] = run_implicit_task(k, req_ptr, lo, hi, priv, rounds[k], A);
  if (checksum) *checksum = checksum_of(N, digest);
  return OR_OK;
}

/* Implicit bodies run in a caller-given order (no dependence checks). */
int or_implicit_in_order(uint32_t N, const uint64_t* req_ptr, const uint64_t* lo,
                         const uint64_t* hi, const uint32_t* priv, const uint32_t* rounds,
                         uint64_t seed, uint64_t space, const uint32_t* order, uint32_t* A,
                         uint32_t* digest, uint64_t* checksum) {
  uint32_t i;
  uint8_t* seen;
  int rc = check_reqs(N, req_ptr, lo, hi, priv, space);
  if (rc != OR_OK) return rc;
  seen = (uint8_t*)calloc((size_t)N + 1, 1);
  if (!seen) return OR_ENOMEM;
  init_array(A, space, seed);
  for (i = 0; i < N; i++) {
    uint32_t k = order[i];
    if (k >= N || seen[k]) { free(seen); return OR_EORDER; }
    seen[k] = 1;
    digest[k] = run_implicit_task(k, req_ptr, lo, hi, priv, rounds[k], A);
  }
  free(seen);
  if (checksum) *checksum = checksum_of(N, digest);
  return OR_OK;
}

static int tasks_conflict(uint32_t j, uint32_t k, const uint64_t* req_ptr, const uint64_t* lo,
                          const uint64_t* hi, const uint32_t* priv) {
  uint64_t a, b;
  for (a = req_ptr[j]; a < req_ptr[j + 1]; a++)
    for (b = req_ptr[k]; b < req_ptr[k + 1]; b++)
      if (overlap(lo[a], hi[a], lo[b], hi[b]) && (priv[a] == OR_RW || priv[b] == OR_RW)) return 1;
  return 0;
}

/*
 * Brute-force conflict DAG: test every pair j<k.  Row j of the CSR lists the
 * successors k of j in ascending order.  cap bounds col; *E receives the edge
 * count (also when it exceeds cap, in which case OR_ENOMEM is returned).
 */
int or_conflict_dag(uint32_t N, const uint64_t* req_ptr, const uint64_t* lo, const uint64_t* hi,
                    const uint32_t* priv, uint64_t* row_ptr, uint32_t* col, uint64_t cap,
                    uint64_t* E) {
  uint32_t j, k;
  uint64_t e = 0;
  row_ptr[0] = 0;
  for (j = 0; j < N; j++) {
    for (k = j + 1; k < N; k++)
      if (tasks_conflict(j, k, req_ptr, lo, hi, priv)) {
        if (e < cap) col[e] = k;
        e++;
      }
    row_ptr[j + 1] = e;
  }
  *E = e;
  return e <= cap ? OR_OK : OR_ENOMEM;
}

/* One row of the brute-force conflict DAG: successors of task j, ascending. */
int or_conflict_row(uint32_t N, const uint64_t* req_ptr, const uint64_t* lo, const uint64_t* hi,
                    const uint32_t* priv, uint32_t j, uint32_t* out, uint64_t cap, uint64_t* cnt) {
  uint32_t k;
  uint64_t e = 0;
  if (j >= N) return OR_EINVAL;
  for (k = j + 1; k < N; k++)
    if (tasks_conflict(j, k, req_ptr, lo, hi, priv)) {
      if (e < cap) out[e] = k;
      e++;
    }
  *cnt = e;
  return e <= cap ? OR_OK : OR_ENOMEM;
}

/* Predecessors of task k in the brute-force conflict DAG, ascending. */
int or_conflict_preds(uint32_t N, const uint64_t* req_ptr, const uint64_t* lo, const uint64_t* hi,
                      const uint32_t* priv, uint32_t k, uint32_t* out, uint64_t cap, uint64_t* cnt) {
  uint32_t j;
  uint64_t e = 0;
  if (k >= N) return OR_EINVAL;
  for (j = 0; j < k; j++)
    if (tasks_conflict(j, k, req_ptr, lo, hi, priv)) {
      if (e < cap) out[e] = j;
      e++;
    }
  *cnt = e;
  return e <= cap ? OR_OK : OR_ENOMEM;
}
