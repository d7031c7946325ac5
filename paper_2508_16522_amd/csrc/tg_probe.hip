// Roofline probes: the denominators of the executor's roofline fractions,
// measured on the device the library runs on.
//   mix rate      : word-rounds/s of a dependency-free kernel running the
//                   task body's mix (the plain integer-VALU peak): the
//                   better of a one-vector-per-lane grid and a persistent
//                   two-vector-per-lane grid;
//   copy bandwidth: HBM bytes/s (read + write) of a streaming copy;
//   atomics       : device-scope u32 atomic decrements per second on
//                   distinct addresses and on one contended address;
//   launch        : back-to-back empty kernel launches per second;
//   hand-off      : latency of one dependent hop between two wavefronts on
//                   different XCDs as the executor makes it (the per-level
//                   floor of a dependence chain): the receiver sees the
//                   sender's signal, loads its 1 KB payload with device-scope
//                   loads, stores its own payload, drains its stores and
//                   signals back with one device atomic.
#include "taskgraph.h"
#include "tg_internal.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The mix at the executor's occupancy: same launch bounds and waves per SIMD.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void p_mix(uint32_t* a, uint32_t rounds) {
  const size_t base = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  u32x4 x = {a[base], a[base + 1], a[base + 2], a[base + 3]};
  for (uint32_t r = 0; r < rounds; ++r) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    x = x * 0x9E3779B1u + 0x7F4A7C15u;
  }
  a[base] = x[0];
  a[base + 1] = x[1];
  a[base + 2] = x[2];
  a[base + 3] = x[3];
}

// The same mix with two 4-word vectors per lane (twice the independent
// chains), in a grid of exactly the co-resident blocks that each loop over
// several chunks, so neither dependent-issue latency nor block turnover
// keeps the VALU idle.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void p_mix8(uint32_t* a, uint32_t rounds,
                                                                                        uint32_t chunks) {
  for (uint32_t c = 0; c < chunks; ++c) {
    const size_t base = (((size_t)c * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x) * 8;
    u32x4 x = {a[base], a[base + 1], a[base + 2], a[base + 3]};
    u32x4 y = {a[base + 4], a[base + 5], a[base + 6], a[base + 7]};
    for (uint32_t r = 0; r < rounds; ++r) {
      x ^= x << 13;
      y ^= y << 13;
      x ^= x >> 17;
      y ^= y >> 17;
      x ^= x << 5;
      y ^= y << 5;
      x = x * 0x9E3779B1u + 0x7F4A7C15u;
      y = y * 0x9E3779B1u + 0x7F4A7C15u;
    }
    a[base] = x[0];
    a[base + 1] = x[1];
    a[base + 2] = x[2];
    a[base + 3] = x[3];
    a[base + 4] = y[0];
    a[base + 5] = y[1];
    a[base + 6] = y[2];
    a[base + 7] = y[3];
  }
}

__global__ __launch_bounds__(256) void p_copy(const u32x4* __restrict__ a, u32x4* __restrict__ b, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ __launch_bounds__(256) void p_atomic_distinct(uint32_t* c, uint32_t mask, uint32_t iters) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t k = 0; k < iters; ++k)
    __hip_atomic_fetch_sub(c + ((i * 2654435761u + k * 40503u) & mask), 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void p_atomic_contended(uint32_t* c, uint32_t iters) {
  if ((threadIdx.x & 63u) == 0)
    for (uint32_t k = 0; k < iters; ++k) __hip_atomic_fetch_sub(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void p_empty() {}

constexpr int kSC1 = 16;  // buffer cache policy: device-scope coherent access

constexpr int kSC0 = 1;   // buffer cache policy: bypass L1, may hit the XCD's L2

// Two single-wave workgroups, blocks ba and bb (workgroup b runs on XCD
// b mod 8), pass a token back and forth `hops` times in total.  A block waits
// for its flag to reach its turn count, reads the other block's 1 KB payload
// (16 bytes per lane), writes its own, drains its stores and increments the
// other block's flag.  Flags are device-scope atomics polled with device-scope
// loads; the payload is accessed at device scope, or (L2PAY, only coherent when
// both blocks share an XCD) through the XCD's L2.  Other blocks exit.  Every
// wait gives up after `spin_cap` polls (status 1).  stamp[0..1]: device clock
// at block ba's first and last hop.
template <bool L2PAY>
__global__ __launch_bounds__(64) void p_handoff(uint32_t* flags, uint32_t* pay, uint32_t hops, uint32_t spin_cap,
                                                uint32_t* status, uint64_t* stamp, uint32_t ba, uint32_t bb) {
  if (blockIdx.x != ba && blockIdx.x != bb) return;
  const uint32_t me = blockIdx.x == ba ? 0u : 1u, other = me ^ 1u, lane = threadIdx.x;
  constexpr int pol = L2PAY ? kSC0 : kSC1;
  const __amdgpu_buffer_rsrc_t mine = __builtin_amdgcn_make_buffer_rsrc(pay + me * 256, 0, 1024, 0x00020000);
  const __amdgpu_buffer_rsrc_t theirs = __builtin_amdgcn_make_buffer_rsrc(pay + other * 256, 0, 1024, 0x00020000);
  u32x4 acc = {lane, 0u, 0u, 0u};
  uint64_t t0 = 0;
  // block ba takes hops 0, 2, 4, ...; block bb hops 1, 3, 5, ...
  for (uint32_t h = me; h < hops; h += 2) {
    const uint32_t turn = h / 2;  // messages this block must have received
    uint32_t spins = 0;
    while (__hip_atomic_load(flags + me * 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < turn + me) {
      if (++spins > spin_cap) {
        if (lane == 0) __hip_atomic_store(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
    }
    if (me == 0 && h == 0) t0 = __builtin_amdgcn_s_memrealtime();
    acc += __builtin_amdgcn_raw_buffer_load_b128(theirs, lane * 16, 0, pol);
    __builtin_amdgcn_raw_buffer_store_b128(acc, mine, lane * 16, 0, pol);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (lane == 0) __hip_atomic_fetch_add(flags + other * 32, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (me == 0 && lane == 0) {
    stamp[0] = t0;
    stamp[1] = __builtin_amdgcn_s_memrealtime();
  }
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  hipError_t start() { return hipEventRecord(a, nullptr); }
  hipError_t stop(float* ms) {
    hipError_t e = hipEventRecord(b, nullptr);
    if (e != hipSuccess) return e;
    if ((e = hipEventSynchronize(b)) != hipSuccess) return e;
    return hipEventElapsedTime(ms, a, b);
  }
};

}  // namespace

extern "C" tg_status tg_probe(uint32_t kind, double* value) {
  if (!value) return TG_EINVAL;
  *value = 0;
  Timer t;
  float ms = 0;
  hipError_t e = hipSuccess;
  void *a = nullptr, *b = nullptr;
  switch (kind) {
    case TG_PROBE_MIX_RATE: {
      // 16M words, 8192 rounds (about 30 ms per launch): a warm-up launch,
      // then the best of five, so the clocks have settled
      const uint32_t threads = 1u << 22, rounds = 8192;
      if ((e = hipMalloc(&a, (size_t)threads * 16)) != hipSuccess) break;
      if ((e = hipMemset(a, 7, (size_t)threads * 16)) != hipSuccess) break;
      hipLaunchKernelGGL(p_mix, dim3(threads / 256), dim3(256), 0, nullptr, (uint32_t*)a, rounds);  // warm
      float best = 1e30f;
      for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) {
        (void)t.start();
        hipLaunchKernelGGL(p_mix, dim3(threads / 256), dim3(256), 0, nullptr, (uint32_t*)a, rounds);
        if ((e = t.stop(&ms)) != hipSuccess) break;
        best = ms < best ? ms : best;
      }
      double rate = 4.0 * threads * rounds / (best * 1e-3);
      // the persistent two-vector variant: 8 co-resident blocks per CU, each
      // thread 8 words per chunk, 4 chunks (the same 16M words in total)
      int dev = 0, cus = 0;
      if ((e = hipGetDevice(&dev)) != hipSuccess) break;
      if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) break;
      const uint32_t blocks = 8u * (uint32_t)cus;
      const uint32_t chunks = (uint32_t)((size_t)threads * 4 / ((size_t)blocks * 256 * 8));
      if (chunks > 0) {
        hipLaunchKernelGGL(p_mix8, dim3(blocks), dim3(256), 0, nullptr, (uint32_t*)a, rounds / 2, chunks);  // warm
        best = 1e30f;
        for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) {
          (void)t.start();
          hipLaunchKernelGGL(p_mix8, dim3(blocks), dim3(256), 0, nullptr, (uint32_t*)a, rounds / 2, chunks);
          if ((e = t.stop(&ms)) != hipSuccess) break;
          best = ms < best ? ms : best;
        }
        const double r8 = 8.0 * blocks * 256.0 * chunks * (rounds / 2) / (best * 1e-3);
        if (r8 > rate) rate = r8;
      }
      *value = rate;
      break;
    }
    case TG_PROBE_HANDOFF_NS:
    case TG_PROBE_HANDOFF_SAME_XCD_NS:
    case TG_PROBE_HANDOFF_FAR_XCD_NS:
    case TG_PROBE_HANDOFF_L2_NS: {
      const uint32_t hops = 20000;
      // blocks 0 and 1: neighbouring XCDs; 0 and 4: the far half of the
      // package; 0 and 8: one XCD
      const uint32_t bb = kind == TG_PROBE_HANDOFF_NS ? 1u : kind == TG_PROBE_HANDOFF_FAR_XCD_NS ? 4u : 8u;
      // flags (one per 128-byte line), status, clock stamps, two 1 KB payloads
      if ((e = hipMalloc(&a, 8192)) != hipSuccess) break;
      if ((e = hipMemset(a, 0, 8192)) != hipSuccess) break;
      uint32_t* w = (uint32_t*)a;
      if (kind == TG_PROBE_HANDOFF_L2_NS)
        hipLaunchKernelGGL(p_handoff<true>, dim3(bb + 1), dim3(64), 0, nullptr, w, w + 1024, hops, 1u << 22, w + 64,
                           (uint64_t*)(w + 96), 0u, bb);
      else
        hipLaunchKernelGGL(p_handoff<false>, dim3(bb + 1), dim3(64), 0, nullptr, w, w + 1024, hops, 1u << 22, w + 64,
                           (uint64_t*)(w + 96), 0u, bb);
      if ((e = hipDeviceSynchronize()) != hipSuccess) break;
      uint32_t status = 0;
      uint64_t stamp[2] = {0, 0};
      if ((e = hipMemcpy(&status, w + 64, 4, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if ((e = hipMemcpy(stamp, w + 96, 16, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if (status != 0 || stamp[1] <= stamp[0]) {
        (void)hipFree(a);
        return TG_ETIMEOUT;
      }
      // block 0's clock spans the start of hop 0 to the end of hop hops - 2
      *value = (double)(stamp[1] - stamp[0]) * 10.0 / (double)(hops - 1);
      break;
    }
    case TG_PROBE_COPY_BW: {
      const size_t bytes = 1ull << 31;
      if ((e = hipMalloc(&a, bytes)) != hipSuccess) break;
      if ((e = hipMalloc(&b, bytes)) != hipSuccess) break;
      if ((e = hipMemset(a, 1, bytes)) != hipSuccess) break;
      float best = 1e30f;
      for (int rep = 0; rep < 4; ++rep) {
        (void)t.start();
        hipLaunchKernelGGL(p_copy, dim3(256 * 16), dim3(256), 0, nullptr, (const u32x4*)a, (u32x4*)b, bytes / 16);
        if ((e = t.stop(&ms)) != hipSuccess) break;
        best = ms < best ? ms : best;
      }
      *value = 2.0 * bytes / (best * 1e-3);
      break;
    }
    case TG_PROBE_ATOMIC_DISTINCT: {
      const uint32_t words = 1u << 24, threads = 1u << 20, iters = 64;
      if ((e = hipMalloc(&a, (size_t)words * 4)) != hipSuccess) break;
      if ((e = hipMemset(a, 0, (size_t)words * 4)) != hipSuccess) break;
      (void)t.start();
      hipLaunchKernelGGL(p_atomic_distinct, dim3(threads / 256), dim3(256), 0, nullptr, (uint32_t*)a, words - 1, iters);
      if ((e = t.stop(&ms)) != hipSuccess) break;
      *value = (double)threads * iters / (ms * 1e-3);
      break;
    }
    case TG_PROBE_ATOMIC_CONTENDED: {
      const uint32_t blocks = 1024, iters = 64;
      if ((e = hipMalloc(&a, 256)) != hipSuccess) break;
      if ((e = hipMemset(a, 0, 256)) != hipSuccess) break;
      (void)t.start();
      hipLaunchKernelGGL(p_atomic_contended, dim3(blocks), dim3(256), 0, nullptr, (uint32_t*)a, iters);
      if ((e = t.stop(&ms)) != hipSuccess) break;
      *value = (double)blocks * 4 * iters / (ms * 1e-3);
      break;
    }
    case TG_PROBE_LAUNCH_RATE: {
      const int n = 20000;
      for (int i = 0; i < 100; ++i) hipLaunchKernelGGL(p_empty, dim3(1), dim3(64), 0, nullptr);
      (void)t.start();
      for (int i = 0; i < n; ++i) hipLaunchKernelGGL(p_empty, dim3(1), dim3(64), 0, nullptr);
      if ((e = t.stop(&ms)) != hipSuccess) break;
      *value = n / (ms * 1e-3);
      break;
    }
    default:
      return TG_EINVAL;
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return e == hipSuccess ? TG_OK : TG_EDEVICE;
}
