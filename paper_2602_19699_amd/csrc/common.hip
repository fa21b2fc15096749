// Small utility kernels: the horizon sort that groups instances of similar
// horizon into the same wavefront (longest first), so that lockstep waves of
// a ragged batch waste few steps and the dispatcher hands out the longest
// work first.
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

hipError_t launch_horizon_sort(const int32_t* dT, int B, int Tmax, int32_t* hist, int32_t* perm, hipStream_t st) {
  const int nb = Tmax + 1;
  const int g = (B + 255) / 256 < 1024 ? (B + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_zero_i32, dim3((nb + 255) / 256), dim3(256), 0, st, hist, nb);
  hipLaunchKernelGGL(k_hist, dim3(g), dim3(256), 0, st, dT, B, Tmax, hist);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, hist, nb);
  hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, st, dT, B, Tmax, hist, perm);
  return hipGetLastError();
}

}  // namespace cbic
