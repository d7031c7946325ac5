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

// bent holds nent entries (counted on the host with the same rule as
// k_bucket_count; the host checks the two totals agree).
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

// In-place exclusive scan of u64 (used recursively for block sums).
static hipError_t scan_u64_inplace(uint64_t* data, uint64_t n, std::vector<void*>& tmp, hipStream_t st) {
  if (n <= 1) {
    if (n == 1) return hipMemsetAsync(data, 0, 8, st);
    return hipSuccess;
  }
  const uint64_t nb = (n + 1023) / 1024;
  void* bs = nullptr;
  hipError_t e = hipMalloc(&bs, nb * 8);
  if (e != hipSuccess) return e;
  tmp.push_back(bs);
  hipLaunchKernelGGL(k_scan_u64_block, dim3((uint32_t)nb), dim3(256), 0, st, data, n, (uint64_t*)bs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (nb > 1) {
    if ((e = scan_u64_inplace((uint64_t*)bs, nb, tmp, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, data, n, (const uint64_t*)bs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// out[0..n] = exclusive scan of in[0..n) with out[n] = total.
static hipError_t scan_counts(const uint32_t* in, uint64_t n, uint64_t* out, hipStream_t st) {
  std::vector<void*> tmp;
  hipError_t e = hipSuccess;
  if (n == 0) {
    e = hipMemsetAsync(out, 0, 8, st);
  } else {
    const uint64_t nb = (n + 1023) / 1024;
    void* bs = nullptr;
    e = hipMalloc(&bs, nb * 8);
    if (e == hipSuccess) {
      tmp.push_back(bs);
      hipLaunchKernelGGL(k_scan_block, dim3((uint32_t)nb), dim3(256), 0, st, in, n, out, (uint64_t*)bs);
      e = hipGetLastError();
      if (e == hipSuccess && nb > 1) {
        e = scan_u64_inplace((uint64_t*)bs, nb, tmp, st);
        if (e == hipSuccess) {
          hipLaunchKernelGGL(k_scan_add, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, out, n, (const uint64_t*)bs);
          e = hipGetLastError();
        }
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, out, n, in);
        e = hipGetLastError();
      }
    }
  }
  hipError_t e2 = hipStreamSynchronize(st);
  for (void* p : tmp) (void)hipFree(p);
  return e != hipSuccess ? e : e2;
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

// Infers the conflict DAG of the n_reqs intervals of N tasks.
hipError_t tg_infer_dag_raw(uint32_t N, const uint64_t* req_ptr_p, const void* reqs_p, uint64_t n_reqs, uint64_t space,
                            InferResult& res, std::string& err) {
  using namespace tg;
  const tg_region_req* reqs = (const tg_region_req*)reqs_p;
  const std::vector<uint64_t> req_ptr(req_ptr_p, req_ptr_p + (size_t)N + 1);
  const uint64_t M = n_reqs;
  res.row_ptr.assign((size_t)N + 1, 0);
  res.col.clear();
  if (N == 0) return hipSuccess;
  // bucket width: the power of two nearest the mean non-empty interval length
  long double tot = 0;
  uint64_t nonempty = 0;
  for (uint64_t a = 0; a < M; ++a)
    if (reqs[a].hi > reqs[a].lo) {
      tot += (long double)(reqs[a].hi - reqs[a].lo);
      nonempty++;
    }
  uint32_t shift = 0;
  if (nonempty) {
    const long double mean = tot / nonempty;
    while (shift < 40 && (long double)(1ull << (shift + 1)) <= mean * 1.41421356L) shift++;
  }
  while (((space + (1ull << shift) - 1) >> shift) > (1ull << 26)) shift++;
  const uint64_t nbuckets = (space + (1ull << shift) - 1) >> shift;
  std::vector<IvDev> iv(M ? M : 1);
  uint64_t nent = 0;  // bucket entries: one per (non-empty interval, bucket it touches)
  for (uint32_t k = 0; k < N; ++k)
    for (uint64_t a = req_ptr[k]; a < req_ptr[k + 1]; ++a) {
      iv[a].lo = reqs[a].lo;
      iv[a].hi = reqs[a].hi;
      iv[a].priv = reqs[a].priv;
      iv[a].task = k;
      if (reqs[a].hi > reqs[a].lo) nent += ((reqs[a].hi - 1) >> shift) - (reqs[a].lo >> shift) + 1;
    }
  // The edge count is read back through one pinned word, allocated once per
  // process (outside the timed region) and shared under a lock.
  static std::mutex pinned_mu;
  static uint64_t* pinned = nullptr;
  {
    std::lock_guard<std::mutex> lk(pinned_mu);
    if (!pinned) {
      void* p = nullptr;
      const hipError_t pe = hipHostMalloc(&p, 64, hipHostMallocDefault);
      if (pe != hipSuccess) {
        err = "hipHostMalloc of the read-back word";
        return pe;
      }
      pinned = (uint64_t*)p;
    }
  }
  hipStream_t st;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) {
    err = "hipStreamCreateWithFlags (an earlier launch may have failed)";
    return e;
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  IvDev* d_iv = nullptr;
  uint64_t *d_req = nullptr, *d_bptr = nullptr, *d_row = nullptr;
  uint32_t *d_bcnt = nullptr, *d_bent = nullptr, *d_rcnt = nullptr, *d_col = nullptr;
  uint64_t E = 0;
  const uint32_t M32 = (uint32_t)M;
  auto cleanup = [&]() {
    (void)hipFree(d_iv); (void)hipFree(d_req); (void)hipFree(d_bptr); (void)hipFree(d_row);
    (void)hipFree(d_bcnt); (void)hipFree(d_bent); (void)hipFree(d_rcnt); (void)hipFree(d_col);
    (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); (void)hipStreamDestroy(st);
  };
#define ICHK(x) do { e = (x); if (e != hipSuccess) { err = #x; cleanup(); return e; } } while (0)
  if (M >= 0xFFFFFFFFull) { err = "too many region requirements"; cleanup(); return hipErrorInvalidValue; }
  ICHK(hipMalloc(&d_iv, iv.size() * sizeof(IvDev)));
  ICHK(hipMalloc(&d_req, req_ptr.size() * 8));
  ICHK(hipMalloc(&d_bcnt, nbuckets * 4));
  ICHK(hipMalloc(&d_bptr, (nbuckets + 1) * 8));
  ICHK(hipMalloc(&d_rcnt, (size_t)N * 4));
  ICHK(hipMalloc(&d_row, ((size_t)N + 1) * 8));
  ICHK(hipMalloc(&d_bent, (nent ? nent : 1) * 4));
  // uploads are ordered on the inference stream itself (the host vectors
  // outlive the final stream synchronisation)
  ICHK(hipMemcpyAsync(d_iv, iv.data(), iv.size() * sizeof(IvDev), hipMemcpyHostToDevice, st));
  ICHK(hipMemcpyAsync(d_req, req_ptr.data(), req_ptr.size() * 8, hipMemcpyHostToDevice, st));
  ICHK(hipEventRecord(e0, st));
  ICHK(hipMemsetAsync(d_bcnt, 0, nbuckets * 4, st));
  if (M32) {
    hipLaunchKernelGGL(k_bucket_count, dim3((M32 + 255) / 256), dim3(256), 0, st, d_iv, M32, shift, d_bcnt);
    ICHK(hipGetLastError());
  }
  ICHK(scan_counts(d_bcnt, nbuckets, d_bptr, st));  // d_bptr[nbuckets] == nent
  ICHK(hipMemsetAsync(d_bcnt, 0, nbuckets * 4, st));
  if (M32) {
    hipLaunchKernelGGL(k_bucket_fill, dim3((M32 + 255) / 256), dim3(256), 0, st, d_iv, M32, shift, d_bptr, d_bcnt, d_bent, nent);
    ICHK(hipGetLastError());
  }
  const uint32_t rblocks = (uint32_t)(((uint64_t)N * 64 + 255) / 256);
  hipLaunchKernelGGL(k_rows<false>, dim3(rblocks), dim3(256), 0, st, d_iv, d_req, N, shift, d_bptr, d_bent, d_rcnt,
                     (const uint64_t*)nullptr, (uint32_t*)nullptr);
  ICHK(hipGetLastError());
  ICHK(scan_counts(d_rcnt, N, d_row, st));
  {
    // ordered after the count pass on the inference stream itself
    std::lock_guard<std::mutex> lk(pinned_mu);
    ICHK(hipMemcpyAsync(pinned, d_row + N, 8, hipMemcpyDeviceToHost, st));
    ICHK(hipMemcpyAsync(pinned + 1, d_bptr + nbuckets, 8, hipMemcpyDeviceToHost, st));
    ICHK(hipStreamSynchronize(st));
    E = pinned[0];
    if (pinned[1] != nent) {
      err = "bucket entry count differs between host and device";
      cleanup();
      return hipErrorUnknown;
    }
  }
  if (E >= 0xFFFFFFFFull) { err = "inferred DAG has too many edges"; cleanup(); return hipErrorInvalidValue; }
  ICHK(hipMalloc(&d_col, (E ? E : 1) * 4));
  hipLaunchKernelGGL(k_rows<true>, dim3(rblocks), dim3(256), 0, st, d_iv, d_req, N, shift, d_bptr, d_bent, d_rcnt,
                     d_row, d_col);
  ICHK(hipGetLastError());
  hipLaunchKernelGGL(k_sort_rows, dim3(N), dim3(256), 0, st, d_row, N, d_col);
  ICHK(hipGetLastError());
  ICHK(hipEventRecord(e1, st));
  ICHK(hipStreamSynchronize(st));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  res.ms = ms;
  res.col.resize(E);
  ICHK(hipMemcpyAsync(res.row_ptr.data(), d_row, ((size_t)N + 1) * 8, hipMemcpyDeviceToHost, st));
  if (E) ICHK(hipMemcpyAsync(res.col.data(), d_col, E * 4, hipMemcpyDeviceToHost, st));
  ICHK(hipStreamSynchronize(st));
  cleanup();
#undef ICHK
  return hipSuccess;
}
