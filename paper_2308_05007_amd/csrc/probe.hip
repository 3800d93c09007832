// Bandwidth probe: the memory pattern of a lattice update without its
// arithmetic or neighbour shifts.  Each thread reads one element (float, or
// half for the 16-bit storage modes) from each of `streams` arrays and
// writes one to each of as many; one launch moves 2 * elem * streams * n
// bytes.  It measures what this GPU's memory system
// delivers to a pattern of that many concurrent read and write streams, the
// ceiling the lattice update's bandwidth is compared with.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rwmi {

// planes: value i of node k at i * n + k; tiled: in tiles of 256 nodes, the
// tile's 256 values of array 0, then of array 1, ... (the distributions'
// two-lattice layout)
__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(__half v) { return __half2float(v); }
template <typename T> __device__ __forceinline__ T from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ __half from_f<__half>(float v) { return __float2half(v); }

template <typename T, int NS, bool TILED>
__global__ void __launch_bounds__(256) k_stream_probe(const T* __restrict__ src, T* __restrict__ dst, uint64_t n) {
  const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t base = TILED ? (uint64_t)blockIdx.x * NS * 256 + threadIdx.x : id;
  const uint64_t step = TILED ? 256 : n;
  float f[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) f[i] = to_f(src[base + i * step]);
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < NS; ++i) acc += f[i];
  // every written value depends on every read one
#pragma unroll
  for (int i = 0; i < NS; ++i) dst[base + i * step] = from_f<T>(f[i] * 0.5f + acc * 1e-3f);
}

template <typename T, int NS>
static hipError_t launch_ns(bool tiled, uint64_t n, const void* src, void* dst, hipStream_t s) {
  const dim3 g((unsigned)(n / 256));
  if (tiled) k_stream_probe<T, NS, true><<<g, 256, 0, s>>>((const T*)src, (T*)dst, n);
  else k_stream_probe<T, NS, false><<<g, 256, 0, s>>>((const T*)src, (T*)dst, n);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(int streams, bool tiled, uint64_t n, const void* src, void* dst, hipStream_t s) {
  switch (streams) {
    case 1: return launch_ns<T, 1>(tiled, n, src, dst, s);
    case 2: return launch_ns<T, 2>(tiled, n, src, dst, s);
    case 4: return launch_ns<T, 4>(tiled, n, src, dst, s);
    case 8: return launch_ns<T, 8>(tiled, n, src, dst, s);
    case 19: return launch_ns<T, 19>(tiled, n, src, dst, s);
    default: return hipErrorInvalidValue;
  }
}

// streams in {1, 2, 4, 8, 19}, elem 4 (float) or 2 (half), n a positive
// multiple of 256 below 2^32
hipError_t launch_stream_probe(int streams, int elem, bool tiled, uint64_t n, const void* src, void* dst,
                               hipStream_t s) {
  if (elem == 4) return launch_t<float>(streams, tiled, n, src, dst, s);
  if (elem == 2) return launch_t<__half>(streams, tiled, n, src, dst, s);
  return hipErrorInvalidValue;
}

}  // namespace rwmi
