// Small utility kernels: the horizon sort that groups instances of similar
// horizon into the same wavefront (longest first), so that lockstep waves of
// a ragged batch waste few steps and the dispatcher hands out the longest
// work first.
#include "dev_common.hpp"
#include "runtime.hpp"

namespace cbic {

// hist[0..Tmax] counts instances per bucket (bucket = Tmax - T, so the
// longest horizons come first); one grid-stride pass with atomics.
__global__ void k_hist(const int32_t* __restrict__ T, int B, int Tmax, int32_t* __restrict__ hist) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x) {
    int t = T[i];
    t = t < 1 ? 1 : (t > Tmax ? Tmax : t);
    atomicAdd(&hist[Tmax - t], 1);
  }
}

// exclusive scan of hist[0..Tmax] in one workgroup (in place)
__global__ void __launch_bounds__(1024) k_scan(int32_t* __restrict__ hist, int nb) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int lo = t * per, hi = lo + per < nb ? lo + per : nb;
  int32_t s = 0;
  for (int i = lo; i < hi; ++i) s += hist[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    const int32_t c = hist[i];
    hist[i] = run;
    run += c;
  }
}

// scatter: cursor per bucket, perm[pos] = instance
__global__ void k_scatter(const int32_t* __restrict__ T, int B, int Tmax, int32_t* __restrict__ cursor,
                          int32_t* __restrict__ perm) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x) {
    int t = T[i];
    t = t < 1 ? 1 : (t > Tmax ? Tmax : t);
    const int pos = atomicAdd(&cursor[Tmax - t], 1);
    perm[pos] = i;
  }
}

__global__ void k_zero_i32(int32_t* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, size_t n, int32_t v) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// dst[i] = src[idx[i]]  (status words of a slot list, for the serving loop)
__global__ void k_gather_u32(const uint32_t* __restrict__ src, const int32_t* __restrict__ idx, int n,
                             uint32_t* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

// inst[slots[i]] = i: finished slots write their outputs to compact rows 0..n-1
__global__ void k_set_index(const int32_t* __restrict__ slots, int n, int32_t* __restrict__ inst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) inst[slots[i]] = i;
}

hipError_t launch_gather_u32(const uint32_t* src, const int32_t* idx, int n, uint32_t* dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_u32, dim3((n + 255) / 256), dim3(256), 0, st, src, idx, n, dst);
  return hipGetLastError();
}

hipError_t launch_set_index(const int32_t* slots, int n, int32_t* inst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_index, dim3((n + 255) / 256), dim3(256), 0, st, slots, n, inst);
  return hipGetLastError();
}

// p[0..n) = v by a kernel (not a memset node, so that captured graphs of a
// solve replay it reliably)
hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t g = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_fill_i32, dim3(unsigned(g)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------- iteration order
// A scheduling heuristic, not part of the method: an instance whose initial
// cost J^0 is higher tends to need more iterations, more so the larger the
// non-convex share of J^0 (the part the clip of eq. 7 replaces by a convex
// model), and a wave (or a workgroup) lasts as long as its slowest instance.
// The iteration launches take the slots grouped by horizon (longest first,
// the order the horizon sort already gave the slots) and, within a horizon,
// by J^0 (highest first) in coarse levels below the batch's largest J^0; in a
// batch of one horizon each level is split by the non-convex share (highest
// first), so that instances of similar expected work share waves.  No result
// depends on the order: every instance's arithmetic is its own.
//
// The warm start writes each slot's key (order_key); one workgroup does the
// rest in shared memory: the largest indexes, a histogram of the buckets, its
// scan and the scatter (shared-memory atomics; the order within a bucket is
// arbitrary).
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 8192;  // shared-memory histogram (32 KB)
constexpr int kOrderKeys = 16384;    // slots whose keys stay in shared memory (64 KB)
constexpr int kOrderOLevels = 32;    // levels of the second key (single-horizon batches)

// levels of J^0 per horizon: quarter octaves below the largest J^0 for a
// batch of one horizon (each split again by the second key), whole octaves
// otherwise, fewer if the horizons need more buckets than the histogram holds
__host__ __device__ inline int order_levels(bool ragged, int Tmax) {
  if (!ragged) return 64;
  const int per = kOrderBuckets / (Tmax + 1);
  return per < 16 ? per : 16;
}

__device__ __forceinline__ int order_level(uint32_t a, uint32_t ref, int nlev) {
  if (!a) return nlev - 1;
  const int d = int(ref) - int(a);
  return d < 0 ? 0 : (d > nlev - 1 ? nlev - 1 : d);
}

// bucket of a key.  Ragged: horizon (longest first), then the J^0 level below
// the largest index refJ (highest first).  One horizon: the J^0 level below
// refJ, then the second key's level below its largest index refO (highest
// first).  The last level of either takes values <= 0.
template <bool RAGGED>
__device__ __forceinline__ int order_bucket(uint32_t key, int Tmax, int nlev, uint32_t refJ, uint32_t refO) {
  if constexpr (RAGGED) return (Tmax - int(key >> 11)) * nlev + order_level(key & 2047u, refJ, nlev);
  else return order_level(key >> 11, refJ, nlev) * kOrderOLevels + order_level(key & 2047u, refO, kOrderOLevels);
}

// horizons must fit the key's 20 bits, and ragged ones a level each in the histogram
bool cost_order_supported(bool ragged, int Tmax) {
  return Tmax < (1 << 20) && (!ragged || order_levels(true, Tmax) >= 1);
}

// exclusive scan of a shared-memory histogram hist[0..nb) by the kOrderThreads
// threads of one workgroup (part: kOrderThreads / 64 entries of shared
// memory): a serial run per thread, an inclusive scan of the threads' sums
// within each wave by shuffles, then the wave totals.  Ends with a barrier.
__device__ __forceinline__ void block_exclusive_scan(int32_t* hist, int nb, int32_t* part) {
  const int t = threadIdx.x;
  const int per = (nb + kOrderThreads - 1) / kOrderThreads;
  const int lo = t * per, hi = lo + per < nb ? lo + per : nb;
  int32_t sum = 0;
  for (int i = lo; i < hi; ++i) sum += hist[i];
  int32_t inc = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t v = __shfl_up(inc, o, 64);
    if ((t & 63) >= o) inc += v;
  }
  if ((t & 63) == 63) part[t >> 6] = inc;
  __syncthreads();
  int32_t wbase = 0;
  for (int w = 0; w < (t >> 6); ++w) wbase += part[w];
  int32_t run = wbase + inc - sum;
  for (int i = lo; i < hi; ++i) {
    const int32_t c = hist[i];
    hist[i] = run;
    run += c;
  }
  __syncthreads();
}

template <bool RAGGED, bool CACHED>
__global__ void __launch_bounds__(kOrderThreads) k_cost_order(const uint32_t* __restrict__ Kin, int B, int Tmax,
                                                               int32_t* __restrict__ order) {
  __shared__ int32_t hist[kOrderBuckets];
  __shared__ uint32_t keys[CACHED ? kOrderKeys : 1];
  __shared__ uint32_t wmax[2][kOrderThreads / 64];
  __shared__ int32_t part[kOrderThreads / 64];
  const int t = threadIdx.x;
  const int nlev = order_levels(RAGGED, Tmax);
  const int nb = RAGGED ? (Tmax + 1) * nlev : nlev * kOrderOLevels;
  auto key_at = [&](int s) -> uint32_t { return Kin[s]; };
  auto key_of = [&](int s) -> uint32_t {
    if constexpr (CACHED) return keys[s];
    else return key_at(s);
  };
  for (int i = t; i < nb; i += kOrderThreads) hist[i] = 0;
  // keys (kept in shared memory when they fit) and the largest indexes: of
  // J^0 (mj) and, for one horizon, of the second key (mo)
  uint32_t mj = 0, mo = 0;
#pragma unroll 8
  for (int s = t; s < B; s += kOrderThreads) {
    const uint32_t k = key_at(s);
    if constexpr (CACHED) keys[s] = k;
    const uint32_t a = RAGGED ? (k & 2047u) : (k >> 11), c = RAGGED ? 0u : (k & 2047u);
    mj = a > mj ? a : mj;
    mo = c > mo ? c : mo;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t v = uint32_t(__shfl_xor(int(mj), o, 64)), u = uint32_t(__shfl_xor(int(mo), o, 64));
    mj = v > mj ? v : mj;
    mo = u > mo ? u : mo;
  }
  if ((t & 63) == 0) {
    wmax[0][t >> 6] = mj;
    wmax[1][t >> 6] = mo;
  }
  __syncthreads();
  uint32_t refJ = 0, refO = 0;
#pragma unroll
  for (int w = 0; w < kOrderThreads / 64; ++w) {
    refJ = wmax[0][w] > refJ ? wmax[0][w] : refJ;
    refO = wmax[1][w] > refO ? wmax[1][w] : refO;
  }
#pragma unroll 4
  for (int s = t; s < B; s += kOrderThreads)
    atomicAdd(&hist[order_bucket<RAGGED>(key_of(s), Tmax, nlev, refJ, refO)], 1);
  __syncthreads();
  block_exclusive_scan(hist, nb, part);
#pragma unroll 4
  for (int s = t; s < B; s += kOrderThreads)
    order[atomicAdd(&hist[order_bucket<RAGGED>(key_of(s), Tmax, nlev, refJ, refO)], 1)] = s;
}

hipError_t launch_cost_order(const uint32_t* keys, int B, int Tmax, bool ragged, int32_t* order, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (!cost_order_supported(ragged, Tmax)) return hipErrorInvalidValue;
  const dim3 g(1), b(kOrderThreads);
  const bool cached = B <= kOrderKeys;
  if (ragged && cached) hipLaunchKernelGGL((k_cost_order<true, true>), g, b, 0, st, keys, B, Tmax, order);
  else if (ragged) hipLaunchKernelGGL((k_cost_order<true, false>), g, b, 0, st, keys, B, Tmax, order);
  else if (cached) hipLaunchKernelGGL((k_cost_order<false, true>), g, b, 0, st, keys, B, Tmax, order);
  else hipLaunchKernelGGL((k_cost_order<false, false>), g, b, 0, st, keys, B, Tmax, order);
  return hipGetLastError();
}


// The horizon sort of a batch whose buckets and per-instance bucket indexes
// fit in shared memory, in one workgroup: the histogram of the buckets
// Tmax - T (T clamped into [1, Tmax]), its scan and the scatter, all on
// shared-memory atomics (the order within a bucket is arbitrary, as in the
// grid-wide version below).
__global__ void __launch_bounds__(kOrderThreads) k_horizon_sort_lds(const int32_t* __restrict__ T, int B, int Tmax,
                                                                     int32_t* __restrict__ perm) {
  __shared__ int32_t hist[kOrderBuckets];
  __shared__ uint16_t bucket[kOrderKeys];
  __shared__ int32_t part[kOrderThreads / 64];
  const int t = threadIdx.x;
  const int nb = Tmax + 1;
  for (int i = t; i < nb; i += kOrderThreads) hist[i] = 0;
  __syncthreads();
#pragma unroll 4
  for (int s = t; s < B; s += kOrderThreads) {
    int h = T[s];
    h = h < 1 ? 1 : (h > Tmax ? Tmax : h);
    bucket[s] = uint16_t(Tmax - h);
    atomicAdd(&hist[Tmax - h], 1);
  }
  __syncthreads();
  block_exclusive_scan(hist, nb, part);
#pragma unroll 4
  for (int s = t; s < B; s += kOrderThreads) perm[atomicAdd(&hist[bucket[s]], 1)] = s;
}

hipError_t launch_horizon_sort(const int32_t* dT, int B, int Tmax, int32_t* hist, int32_t* perm, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (B <= kOrderKeys && Tmax + 1 <= kOrderBuckets) {
    hipLaunchKernelGGL(k_horizon_sort_lds, dim3(1), dim3(kOrderThreads), 0, st, dT, B, Tmax, perm);
    return hipGetLastError();
  }
  const int nb = Tmax + 1;
  const int g = (B + 255) / 256 < 1024 ? (B + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_zero_i32, dim3((nb + 255) / 256), dim3(256), 0, st, hist, nb);
  hipLaunchKernelGGL(k_hist, dim3(g), dim3(256), 0, st, dT, B, Tmax, hist);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, hist, nb);
  hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, st, dT, B, Tmax, hist, perm);
  return hipGetLastError();
}

}  // namespace cbic
