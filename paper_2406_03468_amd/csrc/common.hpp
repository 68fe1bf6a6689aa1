// Internal device/host helpers shared by the HIP kernels of the FOSSILS/SPIR library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FS_WAVE 64

// Return FS_ERR_DEVICE from a host function when a HIP call fails.
#define FS_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) {                            \
      fs_set_last_hip_error(e_, #call, __FILE__, __LINE__); \
      return FS_ERR_DEVICE;                            \
    }                                                  \
  } while (0)

void fs_set_last_hip_error(hipError_t e, const char* what, const char* file, int line);

// A wave-uniform 64-bit value as an opaque scalar (readfirstlane of both halves).
__device__ __forceinline__ int64_t fs_uniform64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Error-free transformations (contraction off: a*b and s+p must round separately).
// two_sum: s + e == a + b exactly.  acc_dot: (s, c) += a * b with the rounding errors of the
// product and of the sum gathered in c (compensated dot product, Ogita-Rump-Oishi Dot2).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}
__device__ __forceinline__ void acc_dot(double& s, double& c, double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  const double pe = fma(a, b, -p);
  double t, e;
  two_sum(s, p, t, e);
  s = t;
  c = c + (e + pe);
}
// Compensated sum over groups of (1<<HI) lanes (as wave_sum_low), returns the rounded total.
template <int HI>
__device__ __forceinline__ double wave_sum_low_comp(double s, double c) {
#pragma clang fp contract(off)
#pragma unroll
  for (int off = 1; off < (1 << HI); off <<= 1) {
    const double s2 = __shfl_xor(s, off, FS_WAVE), c2 = __shfl_xor(c, off, FS_WAVE);
    double t, e;
    two_sum(s, s2, t, e);
    s = t;
    c = c + c2 + e;
  }
  return s + c;
}

// Full-wave sum with butterfly shuffles (every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, FS_WAVE);
  return v;
}

// Sum over the lanes whose lane index differs only in bits [lo, 6): lanes sharing lane % (1<<lo).
template <int LO>
__device__ __forceinline__ double wave_sum_high(double v) {
#pragma unroll
  for (int off = 32; off >= (1 << LO); off >>= 1) v += __shfl_xor(v, off, FS_WAVE);
  return v;
}

// Sum over the lanes whose lane index differs only in bits [0, HI): groups of (1<<HI) lanes.
template <int HI>
__device__ __forceinline__ double wave_sum_low(double v) {
#pragma unroll
  for (int off = 1; off < (1 << HI); off <<= 1) v += __shfl_xor(v, off, FS_WAVE);
  return v;
}

// Deterministic block reduction of one double (fixed shuffle + fixed LDS order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh /* NT/64 doubles */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// Device-side early exit: kernels of an inner iteration return at once when the stop flag is set.
__device__ __forceinline__ bool fs_stopped(const int* stop) { return stop != nullptr && *stop != 0; }

// Grid-wide barrier for kernels launched cooperatively (every work-group co-resident).  A central
// arrival counter and a generation word in device memory: the last work-group to arrive resets
// the counter and advances the generation, the others spin on it.  The agent-scope fences make
// each work-group's earlier global writes visible to the others after the barrier.  The spin is
// bounded: on expiry *err is set and the work-group proceeds, so a broken launch cannot hang.
struct GridBarrier {
  unsigned* count;
  unsigned* gen;
  int* err;
};

__device__ __forceinline__ void grid_barrier(const GridBarrier& b, unsigned nblocks, unsigned& local_gen) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned g = local_gen;
    const unsigned arrived = __hip_atomic_fetch_add(b.count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == nblocks) {
      __hip_atomic_store(b.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(b.gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned long long spins = 0;
      while (__hip_atomic_load(b.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1ull << 26)) {
          __hip_atomic_store(b.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    local_gen = g + 1u;
    __threadfence();
  }
  __syncthreads();
}

// ---- fence-free cross-work-group exchange
// An agent-scope release/acquire on this GPU writes back / invalidates the whole L2 of the XCD
// (the XCD L2s are not coherent with each other), which makes a fenced grid barrier cost 10-20 us
// and evicts the working set.  Data that other work-groups read is instead written and read with
// relaxed agent-scope atomics (coherent accesses that bypass the non-coherent L2 copies), and the
// barrier only orders them: every thread waits for its own stores to complete (s_waitcnt) before
// the work-group arrives, and readers issue their loads after observing the new generation.
// Kernels using grid_barrier_co must route ALL data shared across work-groups through
// st_co / ld_co / st_cob / ld_cob (or re-read only what they wrote themselves).
__device__ __forceinline__ void st_co(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_co(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stores_complete() { __builtin_amdgcn_s_waitcnt(0); }

// Bulk coherent traffic: raw buffer loads/stores with the SC1 cache-policy bit (the same coherence
// as the relaxed agent-scope atomics above, but the compiler keeps many of them in flight instead of
// waiting after each one).  A resource covers `bytes` (< 4 GiB) from `base`; out-of-range offsets
// read 0 / drop the store.  Word 3 is the gfx9 raw-buffer format (32-bit data format).
constexpr int FS_CPOL_SC1 = 16;
constexpr int FS_RSRC_WORD3 = 0x00020000;
typedef unsigned int fs_u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t co_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)(uint32_t)bytes, FS_RSRC_WORD3);
}
__device__ __forceinline__ double ld_cob(__amdgpu_buffer_rsrc_t r, size_t byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(uint32_t)byte_off, 0, FS_CPOL_SC1));
}
__device__ __forceinline__ void st_cob(__amdgpu_buffer_rsrc_t r, size_t byte_off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(fs_u32x2, v), r, (int)(uint32_t)byte_off, 0, FS_CPOL_SC1);
}

// Arrival counters: FS_BAR_SLOTS monotonic counters on separate 128-byte lines (work-group g adds
// to slot g % FS_BAR_SLOTS, so arrivals do not all serialize on one address); barrier number c is
// passed when the slots sum to (c + 1) * nblocks.  Lanes of wave 0 poll one slot each.  No reset
// between barriers: the words are zeroed once before the launch (FS_BAR_WORDS words).
constexpr int FS_BAR_SLOTS = 8;
constexpr int FS_BAR_STRIDE = 32;  // unsigned words per slot (128 bytes)
constexpr int FS_BAR_WORDS = FS_BAR_SLOTS * FS_BAR_STRIDE + 8;
__device__ __forceinline__ void grid_barrier_co(const GridBarrier& b, unsigned nblocks, unsigned& local_gen) {
  stores_complete();
  __syncthreads();
  const unsigned target = (local_gen + 1u) * nblocks;
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(b.count + (blockIdx.x % FS_BAR_SLOTS) * FS_BAR_STRIDE, 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    unsigned long long spins = 0;
    while (true) {
      unsigned v = (lane < FS_BAR_SLOTS)
                       ? __hip_atomic_load(b.count + lane * FS_BAR_STRIDE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       : 0u;
#pragma unroll
      for (int off = 1; off < FS_BAR_SLOTS; off <<= 1) v += __shfl_xor(v, off, FS_WAVE);
      if (__shfl(v, 0, FS_WAVE) >= target) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1ull << 26)) {
        if (lane == 0) __hip_atomic_store(b.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  local_gen += 1u;
  __syncthreads();
}

// Launch a kernel that synchronizes its whole grid with the barriers above as an ordinary dispatch,
// after checking that every work-group can be resident at once (grid <= occupancy x CUs).  The
// HIP cooperative-launch path is not used: on this GPU it serializes against the work of every
// other stream, which would stop the solves of a server's slots from overlapping.  When several
// streams launch such grids, their owners reserve work-groups first (CoopBudget) so that the grids
// running together always fit; ordinary kernels on other streams only delay residency (they finish
// on their own), and the bounded spin of the barriers turns any failure into an error flag.
inline hipError_t fs_launch_resident(const void* fn, dim3 grid, dim3 block, void** args, size_t shmem,
                                     hipStream_t s) {
  int dev = 0, ncu = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, (int)(block.x * block.y * block.z), shmem);
  if (e != hipSuccess) return e;
  if (per < 1 || (int64_t)grid.x * grid.y * grid.z > (int64_t)per * ncu) return hipErrorCooperativeLaunchTooLarge;
  return hipLaunchKernel(fn, grid, block, args, shmem, s);
}

// Zero the barrier words before a cooperative launch (a kernel, so it is also graph-safe).
__global__ void k_barrier_reset(unsigned* words, int n);
