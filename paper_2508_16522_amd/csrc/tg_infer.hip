// Dependence inference for implicitly parallel graphs (device side).
//
// Section 2 and Section 5 of the paper: tasks declare the data they access,
// and the runtime discovers the dependences so that the parallel execution
// equals sequential program order.  The rule applied here: tasks j < k
// conflict iff an interval of j and an interval of k overlap and at least one
// of the two is read-write; every conflicting pair becomes an edge j -> k
// (no transitive reduction, which Section 5 names as the kind of non-linear
// optimisation a compiler may avoid).
//
// Device pipeline (one launch each, all on the caller's stream):
//   1. bucket count   : every non-empty interval is registered in each bucket
//                       of width 2^shift it overlaps (device atomics);
//   2. scan           : exclusive scan of bucket sizes;
//   3. bucket fill    : interval indices written into their buckets;
//   4. row count      : one wavefront per task j scans the buckets of its
//                       intervals and counts its distinct successors k > j;
//   5. scan           : exclusive scan of row sizes -> row_ptr;
//   6. row fill       : the same scan writes the successors;
//   7. row sort       : each row sorted ascending (bitonic, all comparators
//                       ascending so padding never moves).
// Duplicates never arise: an interval pair is counted only in the bucket
// holding the start of its intersection, and a task pair only for its
// lexicographically first conflicting interval pair.
#include "taskgraph.h"
#include "tg_internal.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

namespace tg {

struct alignas(16) IvDev {
  uint64_t lo, hi;
  uint32_t task, priv;
};

// Empty intervals share no element and never conflict.
__device__ __forceinline__ bool iv_conflict(const IvDev& a, const IvDev& b) {
  return a.lo < a.hi && b.lo < b.hi && a.lo < b.hi && b.lo < a.hi && (a.priv == 2u || b.priv == 2u);
}

__global__ void k_bucket_count(const IvDev* iv, uint32_t M, uint32_t shift, uint32_t* bcnt) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= M) return;
  const IvDev x = iv[a];
  if (x.lo >= x.hi) return;
  for (uint64_t b = x.lo >> shift; b <= (x.hi - 1) >> shift; ++b) atomicAdd(bcnt + b, 1u);
}

// bent holds nent entries (the total of the scanned bucket counts).
__global__ void k_bucket_fill(const IvDev* iv, uint32_t M, uint32_t shift, const uint64_t* bptr, uint32_t* bfill,
                              uint32_t* bent, uint64_t nent) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= M) return;
  const IvDev x = iv[a];
  if (x.lo >= x.hi) return;
  for (uint64_t b = x.lo >> shift; b <= (x.hi - 1) >> shift; ++b) {
    const uint32_t slot = atomicAdd(bfill + b, 1u);
    const uint64_t pos = bptr[b] + slot;
    if (pos < nent) bent[pos] = a;
  }
}

// True iff (a, b) is the lexicographically first conflicting interval pair
// of tasks (j, k); a ranges over j's intervals, b over k's.
__device__ __forceinline__ bool first_pair(const IvDev* iv, const uint64_t* req_ptr, uint32_t j, uint32_t k,
                                           uint64_t a, uint64_t b) {
  const uint64_t kb = req_ptr[k], ke = req_ptr[k + 1];
  for (uint64_t a2 = req_ptr[j]; a2 <= a; ++a2) {
    const IvDev x = iv[a2];
    const uint64_t bend = (a2 == a) ? b : ke;
    for (uint64_t b2 = kb; b2 < bend; ++b2)
      if (iv_conflict(x, iv[b2])) return false;
  }
  return true;
}

// Successor scan of row j; FILL = false counts, FILL = true writes col.
template <bool FILL>
__global__ __launch_bounds__(256) void k_rows(const IvDev* iv, const uint64_t* req_ptr, uint32_t N, uint32_t shift,
                                              const uint64_t* bptr, const uint32_t* bent, uint32_t* rowcnt,
                                              const uint64_t* row_ptr, uint32_t* col) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t j = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (j >= N) return;
  uint32_t count = 0;
  uint64_t out = FILL ? row_ptr[j] : 0;
  for (uint64_t a = req_ptr[j]; a < req_ptr[j + 1]; ++a) {
    const IvDev x = iv[a];
    if (x.lo >= x.hi) continue;
    for (uint64_t B = x.lo >> shift; B <= (x.hi - 1) >> shift; ++B) {
      const uint64_t eb = bptr[B], ee = bptr[B + 1];
      for (uint64_t e0 = eb; e0 < ee; e0 += 64) {
        bool hit = false;
        uint32_t k = 0;
        if (e0 + lane < ee) {
          const uint32_t bi = bent[e0 + lane];
          const IvDev y = iv[bi];
          k = y.task;
          if (k > j && iv_conflict(x, y) && (((x.lo > y.lo) ? x.lo : y.lo) >> shift) == B)
            hit = first_pair(iv, req_ptr, j, k, a, bi);
        }
        const uint64_t m = __ballot(hit);
        if (FILL && hit) {
          const uint32_t before = __popcll(m & ((1ull << lane) - 1ull));
          col[out + before] = k;
        }
        const uint32_t c = (uint32_t)__popcll(m);
        count += c;
        out += c;
      }
    }
  }
  if (!FILL && lane == 0) rowcnt[j] = count;
}

// Interval table and input checks, one thread per task: task k's
// requirements rq[req_ptr[k] .. req_ptr[k+1]) become IvDev entries tagged
// with k.  summary[0] += total length of the non-empty intervals,
// summary[1] += their number (one atomic per wavefront), summary[2] |=
// error bits: 1 = row pointers that do not run from 0 up to the interval
// count without decreasing, 2 = an
// interval with lo > hi or beyond the index space, 4 = an unknown privilege,
// 8 = a read-write interval overlapping another interval of its own task.
__global__ __launch_bounds__(256) void k_make_iv(const tg_region_req* rq, const uint64_t* req_ptr, uint32_t N,
                                                 uint64_t M, uint64_t space, IvDev* iv,
                                                 unsigned long long* summary) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long len = 0, cnt = 0;
  uint32_t err = 0;
  if (k < N) {
    const uint64_t b = req_ptr[k], e = req_ptr[k + 1];
    // the rows must partition [0, M): start at 0, never decrease, end at M
    if ((k == 0 && b != 0) || (k == N - 1 && e != M)) err |= 1u;
    if (e < b || e > M) {
      err |= 1u;
    } else {
      for (uint64_t a = b; a < e; ++a) {
        const tg_region_req q = rq[a];
        IvDev x;
        x.lo = q.lo;
        x.hi = q.hi;
        x.task = k;
        x.priv = q.priv;
        iv[a] = x;
        if (q.lo > q.hi || q.hi > space) err |= 2u;
        if (q.priv != TG_RO && q.priv != TG_RW) err |= 4u;
        if (q.hi > q.lo) {
          len += q.hi - q.lo;
          ++cnt;
        }
        for (uint64_t a2 = b; a2 < e; ++a2) {
          if (a2 == a) continue;
          const tg_region_req r = rq[a2];
          if ((q.priv == TG_RW || r.priv == TG_RW) && q.lo < q.hi && r.lo < r.hi && q.lo < r.hi && r.lo < q.hi)
            err |= 8u;
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    len += __shfl_xor(len, o, 64);
    cnt += __shfl_xor(cnt, o, 64);
  }
  if ((threadIdx.x & 63u) == 0) {
    atomicAdd(summary + 0, len);
    atomicAdd(summary + 1, cnt);
  }
  if (err) atomicOr((unsigned int*)(summary + 2), err);
}

// ---------------------------------------------------------------- scan

// Exclusive scan of u32 counts into u64 offsets (out has n+1 entries).
__global__ __launch_bounds__(256) void k_scan_block(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* bsum) {
  __shared__ uint64_t s[256];
  const uint64_t base = (uint64_t)blockIdx.x * 1024;
  uint64_t v[4], t = 0;
  for (int i = 0; i < 4; ++i) {
    const uint64_t idx = base + threadIdx.x * 4 + i;
    v[i] = idx < n ? in[idx] : 0;
    t += v[i];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (uint32_t o = 1; o < 256; o <<= 1) {
    const uint64_t add = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  uint64_t run = s[threadIdx.x] - t;
  for (int i = 0; i < 4; ++i) {
    const uint64_t idx = base + threadIdx.x * 4 + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = s[255];
}

__global__ __launch_bounds__(256) void k_scan_u64_block(uint64_t* data, uint64_t n, uint64_t* bsum) {
  __shared__ uint64_t s[256];
  const uint64_t base = (uint64_t)blockIdx.x * 1024;
  uint64_t v[4], t = 0;
  for (int i = 0; i < 4; ++i) {
    const uint64_t idx = base + threadIdx.x * 4 + i;
    v[i] = idx < n ? data[idx] : 0;
    t += v[i];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (uint32_t o = 1; o < 256; o <<= 1) {
    const uint64_t add = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  uint64_t run = s[threadIdx.x] - t;
  for (int i = 0; i < 4; ++i) {
    const uint64_t idx = base + threadIdx.x * 4 + i;
    if (idx < n) data[idx] = run;
    run += v[i];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = s[255];
}

__global__ void k_scan_add(uint64_t* out, uint64_t n, const uint64_t* boff) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) out[idx] += boff[idx / 1024];
}

__global__ void k_scan_total(uint64_t* out, uint64_t n, const uint32_t* in) {
  // out[n] = out[n-1] + in[n-1]
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = n ? out[n - 1] + in[n - 1] : 0;
}

// Device memory of one inference: allocated with hipMalloc (freed when the
// workspace goes away), or carved in order from a fixed region (the
// allocation-free entry point's scratch array), in which case a request
// that does not fit fails and names the array.
struct Workspace {
  uint8_t* base = nullptr;  // fixed region; null: allocate
  size_t cap = 0, used = 0;
  std::vector<void*> owned;
  const char* missing = nullptr;  // array that did not fit the fixed region
  Workspace() = default;
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  ~Workspace() {
    for (void* p : owned) (void)hipFree(p);
  }
  hipError_t get(size_t bytes, const char* name, void** out) {
    bytes = bytes ? (bytes + 255) & ~(size_t)255 : 256;
    if (base) {
      if (bytes > cap - used) {
        missing = name;
        return hipErrorOutOfMemory;
      }
      *out = base + used;
      used += bytes;
      return hipSuccess;
    }
    const hipError_t e = hipMalloc(out, bytes);
    if (e == hipSuccess) owned.push_back(*out);
    return e;
  }
};

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Clears device words with a kernel (callers may record the work into a HIP
// graph, where memset nodes are avoided).
static hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// In-place exclusive scan of u64 (used recursively for block sums).
static hipError_t scan_u64_inplace(uint64_t* data, uint64_t n, Workspace& ws, hipStream_t st) {
  if (n <= 1) return n == 1 ? fill_u32((uint32_t*)data, 2, 0, st) : hipSuccess;
  const uint64_t nb = (n + 1023) / 1024;
  void* bs = nullptr;
  hipError_t e = ws.get(nb * 8, "scan partial sums", &bs);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_u64_block, dim3((uint32_t)nb), dim3(256), 0, st, data, n, (uint64_t*)bs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (nb > 1) {
    if ((e = scan_u64_inplace((uint64_t*)bs, nb, ws, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, data, n, (const uint64_t*)bs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// out[0..n] = exclusive scan of in[0..n) with out[n] = total (stream-ordered).
static hipError_t scan_counts(const uint32_t* in, uint64_t n, uint64_t* out, Workspace& ws, hipStream_t st) {
  if (n == 0) return fill_u32((uint32_t*)out, 2, 0, st);
  const uint64_t nb = (n + 1023) / 1024;
  void* bs = nullptr;
  hipError_t e = ws.get(nb * 8, "scan partial sums", &bs);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_block, dim3((uint32_t)nb), dim3(256), 0, st, in, n, out, (uint64_t*)bs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (nb > 1) {
    if ((e = scan_u64_inplace((uint64_t*)bs, nb, ws, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, out, n, (const uint64_t*)bs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, out, n, in);
  return hipGetLastError();
}

// ------------------------------------------------------------- row sort

constexpr uint32_t kSortLds = 8192;  // words staged in LDS per row

__device__ __forceinline__ void cswap_lds(uint32_t* a, uint32_t i, uint32_t j) {
  const uint32_t x = a[i], y = a[j];
  if (y < x) {
    a[i] = y;
    a[j] = x;
  }
}

// Ascending bitonic network over a virtual array padded to a power of two
// with +infinity; every comparator puts the minimum at the lower index, so
// comparators touching the padding are no-ops and are skipped.
__global__ __launch_bounds__(1024) void k_sort_rows(const uint64_t* row_ptr, uint32_t N, uint32_t* col) {
  __shared__ uint32_t s[kSortLds];
  const uint32_t row = blockIdx.x;
  if (row >= N) return;
  const uint64_t b = row_ptr[row];
  const uint32_t L = (uint32_t)(row_ptr[row + 1] - b);
  if (L < 2) return;
  uint32_t P = 1;
  while (P < L) P <<= 1;
  if (L <= kSortLds) {
    for (uint32_t i = threadIdx.x; i < L; i += blockDim.x) s[i] = col[b + i];
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
      // flip step
      for (uint32_t i = threadIdx.x; i < P / 2; i += blockDim.x) {
        const uint32_t blk = i / (k / 2), off = i % (k / 2);
        const uint32_t lo = blk * k + off, hi = blk * k + k - 1 - off;
        if (hi < L) cswap_lds(s, lo, hi);
      }
      __syncthreads();
      for (uint32_t h = k / 4; h >= 1; h >>= 1) {
        for (uint32_t i = threadIdx.x; i < P / 2; i += blockDim.x) {
          const uint32_t blk = i / h, off = i % h;
          const uint32_t lo = blk * 2 * h + off, hi = lo + h;
          if (hi < L) cswap_lds(s, lo, hi);
        }
        __syncthreads();
      }
    }
    for (uint32_t i = threadIdx.x; i < L; i += blockDim.x) col[b + i] = s[i];
  } else {
    uint32_t* a = col + b;
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t i = threadIdx.x; i < P / 2; i += blockDim.x) {
        const uint32_t blk = i / (k / 2), off = i % (k / 2);
        const uint32_t lo = blk * k + off, hi = blk * k + k - 1 - off;
        if (hi < L) {
          const uint32_t x = __hip_atomic_load(a + lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint32_t y = __hip_atomic_load(a + hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (y < x) {
            __hip_atomic_store(a + lo, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(a + hi, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      for (uint32_t h = k / 4; h >= 1; h >>= 1) {
        for (uint32_t i = threadIdx.x; i < P / 2; i += blockDim.x) {
          const uint32_t blk = i / h, off = i % h;
          const uint32_t lo = blk * 2 * h + off, hi = lo + h;
          if (hi < L) {
            const uint32_t x = __hip_atomic_load(a + lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t y = __hip_atomic_load(a + hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (y < x) {
              __hip_atomic_store(a + lo, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              __hip_atomic_store(a + hi, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
    }
  }
}

// ------------------------------------------------------- initial array

__global__ void k_init_data(uint32_t* A, uint64_t space, uint64_t key2) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < space; e += stride) {
    uint64_t z = key2 ^ e;
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    A[e] = (uint32_t)(z ^ (z >> 31));
  }
}

}  // namespace tg

hipError_t tg_launch_init_data(uint32_t* A, uint64_t space, uint64_t key2, hipStream_t s) {
  uint64_t blocks = (space + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(tg::k_init_data, dim3((uint32_t)blocks), dim3(256), 0, s, A, space, key2);
  return hipGetLastError();
}

// ------------------------------------------------------------ host driver

namespace {

using tg::IvDev;
using tg::Workspace;

// Bucket width 2^shift: the power of two nearest the mean non-empty interval
// length, widened until the index space needs at most max_buckets buckets.
uint32_t choose_shift(unsigned long long total_len, unsigned long long nonempty, uint64_t space,
                      uint64_t max_buckets) {
  uint32_t shift = 0;
  if (nonempty) {
    const long double mean = (long double)total_len / (long double)nonempty;
    while (shift < 40 && (long double)(1ull << (shift + 1)) <= mean * 1.41421356L) shift++;
  }
  while (((space + (1ull << shift) - 1) >> shift) > max_buckets) shift++;
  return shift;
}

// Copies `bytes` of device memory to host memory on `st` and waits: through
// the pinned staging word when one is given, else straight into `host`.
hipError_t read_back(void* host, const void* dev, size_t bytes, uint64_t* pinned, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(pinned ? (void*)pinned : host, dev, bytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && pinned) memcpy(host, pinned, bytes);
  return e;
}

// Inference proper, on device inputs, all work ordered on `st`:
//   rq[M], req_ptr[N+1] : the requirements (device);
//   row[N+1]            : receives the out-edge row pointers (device);
//   *col                : receives the successors: when alloc_col is set a
//                         buffer of the exact size is taken from the
//                         workspace, else *col (capacity col_cap) is used
//                         and a larger edge count fails with TG_ENOMEM;
//   *E                  : the edge count (set also on TG_ENOMEM).
// Returns when the DAG is complete on the device.
tg_status infer_core(Workspace& ws, uint32_t N, uint64_t M, uint64_t space, const tg_region_req* rq,
                     const uint64_t* req_ptr, uint64_t max_buckets, hipStream_t st, uint64_t* pinned,
                     uint64_t* row, uint32_t** col, bool alloc_col, uint64_t col_cap, uint64_t* E) {
  hipError_t e;
#define ICHK(x, what)                                                                                   \
  do {                                                                                                  \
    e = (x);                                                                                            \
    if (e != hipSuccess) {                                                                              \
      if (ws.missing)                                                                                   \
        return tg_set_error(TG_ENOMEM, "dependence inference: the %s do not fit the %zu-byte scratch array", \
                            ws.missing, ws.cap);                                                        \
      return tg_set_error(TG_EDEVICE, "dependence inference (%s): %s", what, hipGetErrorString(e));     \
    }                                                                                                   \
  } while (0)
  *E = 0;
  if (M >= 0xFFFFFFFFull) return tg_set_error(TG_EINVAL, "too many region requirements");
  const uint32_t M32 = (uint32_t)M;
  IvDev* iv = nullptr;
  unsigned long long* summary = nullptr;
  ICHK(ws.get(M * sizeof(IvDev), "intervals", (void**)&iv), "interval table");
  ICHK(ws.get(64, "summary", (void**)&summary), "summary");
  ICHK(tg::fill_u32((uint32_t*)summary, 16, 0, st), "clear");
  hipLaunchKernelGGL(tg::k_make_iv, dim3((N + 255) / 256), dim3(256), 0, st, rq, req_ptr, N, M, space, iv, summary);
  ICHK(hipGetLastError(), "k_make_iv");
  unsigned long long sum[3] = {0, 0, 0};
  ICHK(read_back(sum, summary, sizeof(sum), pinned, st), "summary read-back");
  if (sum[2]) {
    const uint32_t b = (uint32_t)sum[2];
    return tg_set_error(TG_EINVAL, "region requirements: %s%s%s%s",
                        (b & 1) ? "row pointers do not run from 0 to the requirement count without decreasing; " : "",
                        (b & 2) ? "interval with lo > hi or outside the index space; " : "",
                        (b & 4) ? "unknown privilege; " : "",
                        (b & 8) ? "read-write interval overlapping another interval of its task" : "");
  }
  const uint32_t shift = choose_shift(sum[0], sum[1], space, max_buckets);
  const uint64_t nb = (space + (1ull << shift) - 1) >> shift;
  uint32_t* bcnt = nullptr;
  uint64_t* bptr = nullptr;
  ICHK(ws.get(nb * 4, "bucket counts", (void**)&bcnt), "bucket counts");
  ICHK(ws.get((nb + 1) * 8, "bucket offsets", (void**)&bptr), "bucket offsets");
  ICHK(tg::fill_u32(bcnt, nb, 0, st), "clear");
  if (M32) {
    hipLaunchKernelGGL(tg::k_bucket_count, dim3((M32 + 255) / 256), dim3(256), 0, st, iv, M32, shift, bcnt);
    ICHK(hipGetLastError(), "k_bucket_count");
  }
  ICHK(tg::scan_counts(bcnt, nb, bptr, ws, st), "bucket scan");
  uint64_t nent = 0;
  ICHK(read_back(&nent, bptr + nb, 8, pinned, st), "bucket total read-back");
  uint32_t* bent = nullptr;
  ICHK(ws.get(nent * 4, "bucket entries", (void**)&bent), "bucket entries");
  ICHK(tg::fill_u32(bcnt, nb, 0, st), "clear");
  if (M32) {
    hipLaunchKernelGGL(tg::k_bucket_fill, dim3((M32 + 255) / 256), dim3(256), 0, st, iv, M32, shift, bptr, bcnt, bent,
                       nent);
    ICHK(hipGetLastError(), "k_bucket_fill");
  }
  uint32_t* rcnt = nullptr;
  ICHK(ws.get((size_t)N * 4, "row counts", (void**)&rcnt), "row counts");
  const uint32_t rblocks = (uint32_t)(((uint64_t)N * 64 + 255) / 256);
  hipLaunchKernelGGL(tg::k_rows<false>, dim3(rblocks), dim3(256), 0, st, iv, req_ptr, N, shift, bptr, bent, rcnt,
                     (const uint64_t*)nullptr, (uint32_t*)nullptr);
  ICHK(hipGetLastError(), "k_rows (count)");
  ICHK(tg::scan_counts(rcnt, N, row, ws, st), "row scan");
  ICHK(read_back(E, row + N, 8, pinned, st), "edge count read-back");
  if (*E >= 0xFFFFFFFFull) return tg_set_error(TG_EINVAL, "inferred DAG has too many edges (%llu)", (unsigned long long)*E);
  if (alloc_col) {
    ICHK(ws.get(*E * 4, "edges", (void**)col), "edge array");
  } else if (*E > col_cap) {
    return tg_set_error(TG_ENOMEM, "inferred DAG has %llu edges, capacity %llu", (unsigned long long)*E,
                        (unsigned long long)col_cap);
  }
  if (*E) {
    hipLaunchKernelGGL(tg::k_rows<true>, dim3(rblocks), dim3(256), 0, st, iv, req_ptr, N, shift, bptr, bent, rcnt, row,
                       *col);
    ICHK(hipGetLastError(), "k_rows (fill)");
    hipLaunchKernelGGL(tg::k_sort_rows, dim3(N), dim3(256), 0, st, row, N, *col);
    ICHK(hipGetLastError(), "k_sort_rows");
  }
  ICHK(hipStreamSynchronize(st), "inference");
#undef ICHK
  return TG_OK;
}

}  // namespace

// Finalize path: requirements from host memory, DAG back to host memory;
// device buffers allocated for the call.  The edge count and the two other
// small counts come back through one pinned staging buffer, allocated once
// per process (outside any timed region) and shared under a lock.
tg_status tg_infer_dag_host(uint32_t N, const uint64_t* req_ptr, const void* reqs, uint64_t M, uint64_t space,
                            InferResult& res) {
  res.row_ptr.assign((size_t)N + 1, 0);
  res.col.clear();
  res.ms = 0;
  if (N == 0) return TG_OK;
  static std::mutex pinned_mu;
  static uint64_t* pinned = nullptr;
  std::lock_guard<std::mutex> lk(pinned_mu);
  if (!pinned) {
    void* p = nullptr;
    const hipError_t pe = hipHostMalloc(&p, 64, hipHostMallocDefault);
    if (pe != hipSuccess) return tg_set_error(TG_EDEVICE, "hipHostMalloc of the read-back buffer: %s", hipGetErrorString(pe));
    pinned = (uint64_t*)p;
  }
  hipStream_t st = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return tg_set_error(TG_EDEVICE, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  tg_status s = TG_OK;
  // The device memory of the finalize-time inferences is one region kept
  // from call to call (under the lock above) and regrown, by half again,
  // when an inference does not fit: allocating and freeing it per call cost
  // more than the inference kernels.
  static void* region = nullptr;
  static size_t region_bytes = 0;
  for (int attempt = 0;; ++attempt) {
    Workspace ws;
    ws.base = (uint8_t*)region;
    ws.cap = region_bytes;
    tg_region_req* d_rq = nullptr;
    uint64_t *d_req = nullptr, *d_row = nullptr;
    uint32_t* d_col = nullptr;
    uint64_t E = 0;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess ||
        (e = ws.get(M * sizeof(tg_region_req), "requirements", (void**)&d_rq)) != hipSuccess ||
        (e = ws.get(((size_t)N + 1) * 8, "row pointers", (void**)&d_req)) != hipSuccess ||
        (e = ws.get(((size_t)N + 1) * 8, "rows", (void**)&d_row)) != hipSuccess ||
        (M && (e = hipMemcpyAsync(d_rq, reqs, M * sizeof(tg_region_req), hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (e = hipMemcpyAsync(d_req, req_ptr, ((size_t)N + 1) * 8, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipEventRecord(e0, st)) != hipSuccess) {
      s = ws.missing ? TG_ENOMEM : tg_set_error(TG_EDEVICE, "dependence inference set-up: %s", hipGetErrorString(e));
    } else {
      s = infer_core(ws, N, M, space, d_rq, d_req, 1ull << 26, st, pinned, d_row, &d_col, true, 0, &E);
    }
    if (s == TG_ENOMEM && ws.missing && attempt < 8) {
      // the region was too small: wait for the stream, regrow, start again
      (void)hipStreamSynchronize(st);
      const size_t want = std::max<size_t>(ws.used + (size_t(64) << 20), region_bytes + region_bytes / 2);
      if (region) (void)hipFree(region);
      region = nullptr;
      region_bytes = 0;
      if ((e = hipMalloc(&region, want)) != hipSuccess) {
        region = nullptr;
        s = tg_set_error(TG_ENOMEM, "dependence inference: hipMalloc(%zu): %s", want, hipGetErrorString(e));
        break;
      }
      region_bytes = want;
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      e0 = e1 = nullptr;
      continue;
    }
    if (s == TG_OK) {
      res.col.resize(E);
      if ((e = hipEventRecord(e1, st)) != hipSuccess ||
          (e = hipMemcpyAsync(res.row_ptr.data(), d_row, ((size_t)N + 1) * 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (E && (e = hipMemcpyAsync(res.col.data(), d_col, E * 4, hipMemcpyDeviceToHost, st)) != hipSuccess) ||
          (e = hipStreamSynchronize(st)) != hipSuccess) {
        s = tg_set_error(TG_EDEVICE, "dependence inference read-back: %s", hipGetErrorString(e));
      } else {
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) res.ms = ms;
      }
    }
    (void)hipStreamSynchronize(st);
    break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  return s;
}

// ------------------------------------------- inference on device arrays

namespace {

tg_status infer_args(uint32_t N, const uint64_t* req_ptr, const tg_region_req* reqs, uint64_t M, uint64_t* row_ptr,
                     uint32_t* col, uint64_t col_cap, uint64_t* E) {
  if (!E) return tg_set_error(TG_EINVAL, "num_edges is NULL");
  *E = 0;
  if (!req_ptr || !row_ptr) return tg_set_error(TG_EINVAL, "req_ptr and row_ptr must be device arrays of ntasks + 1 words");
  if (M && !reqs) return tg_set_error(TG_EINVAL, "reqs is NULL but nreqs is %llu", (unsigned long long)M);
  if (col_cap && !col) return tg_set_error(TG_EINVAL, "col is NULL but col_cap is %llu", (unsigned long long)col_cap);
  // one workgroup per row sorts the rows: the grid limit bounds the task count
  if (N > 0x7FFFFFFFu) return tg_set_error(TG_EINVAL, "ntasks %u exceeds 2^31 - 1", N);
  return TG_OK;
}

// ntasks = 0: the DAG is one row pointer, 0.
tg_status infer_empty(uint64_t* row_ptr, hipStream_t st) {
  hipError_t e = tg::fill_u32((uint32_t*)row_ptr, 2, 0, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return tg_set_error(TG_EDEVICE, "dependence inference: %s", hipGetErrorString(e));
  return TG_OK;
}

}  // namespace

tg_status tg_infer_dag(uint32_t ntasks, const uint64_t* req_ptr, const tg_region_req* reqs, uint64_t nreqs,
                       uint64_t index_space, uint64_t* row_ptr, uint32_t* col, uint64_t col_cap, uint64_t* num_edges,
                       void* stream) {
  tg_status s = infer_args(ntasks, req_ptr, reqs, nreqs, row_ptr, col, col_cap, num_edges);
  if (s != TG_OK) return s;
  const hipStream_t st = (hipStream_t)stream;
  if (ntasks == 0) return infer_empty(row_ptr, st);
  Workspace ws;
  uint32_t* c = col;
  return infer_core(ws, ntasks, nreqs, index_space, reqs, req_ptr, 1ull << 26, st, nullptr, row_ptr, &c, false,
                    col_cap, num_edges);
}

// ------------------------------------------- allocation-free inference
//
// tg_infer_dag_noalloc takes every temporary of infer_core from one array
// of device memory that the code object defines, so the call makes no
// allocation.  Each device holds its own copy of the array until the process
// ends.  On the host, `scratch` names only a stand-in for the device symbol:
// its device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is handed to kernels and
// copies.

constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
constexpr uint64_t kNoallocMaxBuckets = 1ull << 18;  // bucket arrays of at most 3 MiB

struct ScratchDev {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
  std::mutex mu;  // one call at a time per device in this process
};
ScratchDev g_scratch[kMaxDevices];

size_t round256(uint64_t b) { return (size_t)((b + 255) & ~255ull); }

}  // namespace

tg_status tg_infer_dag_noalloc(uint32_t ntasks, const uint64_t* req_ptr, const tg_region_req* reqs, uint64_t nreqs,
                               uint64_t index_space, uint64_t* row_ptr, uint32_t* col, uint64_t col_cap,
                               uint64_t* num_edges, void* stream) {
  tg_status s = infer_args(ntasks, req_ptr, reqs, nreqs, row_ptr, col, col_cap, num_edges);
  if (s != TG_OK) return s;
  // the interval table, the summary and the row counts must fit before any
  // device work starts; later arrays are checked as they are carved
  const uint64_t need = round256(nreqs * sizeof(IvDev)) + 256 + round256((uint64_t)ntasks * 4);
  if (nreqs > kScratchBytes || need > kScratchBytes)
    return tg_set_error(TG_ENOMEM,
                        "allocation-free inference: %u tasks with %llu requirements need more than the %zu-byte "
                        "scratch array (at least %llu bytes)",
                        ntasks, (unsigned long long)nreqs, kScratchBytes, (unsigned long long)need);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return tg_set_error(TG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return tg_set_error(TG_EDEVICE, "device %d: the scratch table holds devices 0..%d", dev, kMaxDevices - 1);
  ScratchDev& sd = g_scratch[dev];
  std::call_once(sd.once, [&sd] { sd.err = hipGetSymbolAddress(&sd.ptr, HIP_SYMBOL(scratch)); });
  if (sd.err != hipSuccess || !sd.ptr)
    return tg_set_error(TG_EDEVICE, "hipGetSymbolAddress of the scratch array on device %d: %s", dev,
                        hipGetErrorString(sd.err));
  std::lock_guard<std::mutex> lk(sd.mu);
  const hipStream_t st = (hipStream_t)stream;
  if (ntasks == 0) return infer_empty(row_ptr, st);
  Workspace ws;
  ws.base = (uint8_t*)sd.ptr;
  ws.cap = kScratchBytes;
  uint32_t* c = col;
  return infer_core(ws, ntasks, nreqs, index_space, reqs, req_ptr, kNoallocMaxBuckets, st, nullptr, row_ptr, &c, false,
                    col_cap, num_edges);
}
