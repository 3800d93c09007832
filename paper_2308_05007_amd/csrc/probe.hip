// Bandwidth probe: the memory pattern of a lattice update without its
// arithmetic or neighbour shifts.  Each thread reads one float from each of
// `streams` arrays and writes one float to each of as many; one launch
// moves 8 * streams * n bytes.  It measures what this GPU's memory system
// delivers to a pattern of that many concurrent read and write streams, the
// ceiling the lattice update's bandwidth is compared with.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rwmi {

// planes: value i of node k at i * n + k; tiled: in tiles of 256 nodes, the
// tile's 256 values of array 0, then of array 1, ... (the distributions'
// two-lattice layout)
template <int NS, bool TILED>
__global__ void __launch_bounds__(256) k_stream_probe(const float* __restrict__ src, float* __restrict__ dst,
                                                      uint64_t n) {
  const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t base = TILED ? (uint64_t)blockIdx.x * NS * 256 + threadIdx.x : id;
  const uint64_t step = TILED ? 256 : n;
  float f[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) f[i] = src[base + i * step];
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < NS; ++i) acc += f[i];
  // every written value depends on every read one
#pragma unroll
  for (int i = 0; i < NS; ++i) dst[base + i * step] = f[i] * 0.5f + acc * 1e-3f;
}

template <int NS>
static hipError_t launch_ns(bool tiled, uint64_t n, const float* src, float* dst, hipStream_t s) {
  const dim3 g((unsigned)(n / 256));
  if (tiled) k_stream_probe<NS, true><<<g, 256, 0, s>>>(src, dst, n);
  else k_stream_probe<NS, false><<<g, 256, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

// streams in {1, 2, 4, 8, 19}, n a positive multiple of 256 below 2^32
hipError_t launch_stream_probe(int streams, bool tiled, uint64_t n, const float* src, float* dst, hipStream_t s) {
  switch (streams) {
    case 1: return launch_ns<1>(tiled, n, src, dst, s);
    case 2: return launch_ns<2>(tiled, n, src, dst, s);
    case 4: return launch_ns<4>(tiled, n, src, dst, s);
    case 8: return launch_ns<8>(tiled, n, src, dst, s);
    case 19: return launch_ns<19>(tiled, n, src, dst, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rwmi
