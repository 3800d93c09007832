// Host-side launchers of the kernels (defined in k_fp64.hip and k_lowp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "step_map.h"

namespace rwmi {
struct DomView;

// One fused step launch (walker, prologue and fluid blocks; step_map.h) with
// bs threads per block; the grid size follows from a.nb and a.flags.
hipError_t launch_step_p64(int bs, const StepArgs& a, hipStream_t s);
hipError_t launch_step_lowp(int prec, int bs, const StepArgs& a, hipStream_t s);
hipError_t launch_init_p64(const DomView* v, int dom, int64_t N, const double u0[3], hipStream_t s);
hipError_t launch_init_lowp(int prec, const DomView* v, int dom, int64_t N, const double u0[3], hipStream_t s);
hipError_t launch_read_f_p64(const DomView* v, int dom, int64_t N, double* out, hipStream_t s);
hipError_t launch_read_f_lowp(int prec, const DomView* v, int dom, int64_t N, double* out, hipStream_t s);

// precision 0 is FP64 (rwmi::P64)
// Link pass of interpolated bounce-back (k_ibb_links) for the fluid update
// of launch j of a group (none if `blocks`, the fluid blocks, is 0).
hipError_t launch_ibb_links_p64(const DomView* v, int dom, int32_t j, bool dem, unsigned blocks, hipStream_t s);
hipError_t launch_ibb_links_lowp(int prec, const DomView* v, int dom, int32_t j, bool dem, unsigned blocks,
                                 hipStream_t s);
inline hipError_t launch_ibb_links(int prec, const DomView* v, int dom, int32_t j, bool dem, unsigned blocks,
                                   hipStream_t s) {
  return prec == 0 ? launch_ibb_links_p64(v, dom, j, dem, blocks, s)
                   : launch_ibb_links_lowp(prec, v, dom, j, dem, blocks, s);
}
inline hipError_t launch_step(int prec, int bs, const StepArgs& a, hipStream_t s) {
  return prec == 0 ? launch_step_p64(bs, a, s) : launch_step_lowp(prec, bs, a, s);
}
inline hipError_t launch_init(int prec, const DomView* v, int dom, int64_t N, const double u0[3], hipStream_t s) {
  return prec == 0 ? launch_init_p64(v, dom, N, u0, s) : launch_init_lowp(prec, v, dom, N, u0, s);
}
inline hipError_t launch_read_f(int prec, const DomView* v, int dom, int64_t N, double* out, hipStream_t s) {
  return prec == 0 ? launch_read_f_p64(v, dom, N, out, s) : launch_read_f_lowp(prec, v, dom, N, out, s);
}
hipError_t launch_seed(int prec, const DomView* v, int dom, int kind, const double c[3], double sigma, int axis,
                       double lo, double hi, const double* xyz, int64_t n, int attempts, int32_t* cell, void* off,
                       uint8_t* flag, hipStream_t s);
hipError_t launch_seed_scatter(int prec, const DomView* v, int dom, int64_t n, const int32_t* cell, const void* off,
                               const uint8_t* flag, const int32_t* pos, int64_t m, hipStream_t s);
hipError_t launch_occupancy(const DomView* v, int dom, uint32_t* occ, int64_t N, int64_t nw, hipStream_t s);
// walkers per layer along `axis` (n_layers = n[axis] counts, cleared first)
hipError_t launch_profile(const DomView* v, int dom, int axis, int n_layers, int64_t nw, uint32_t* counts,
                          hipStream_t s);
// partial buffers: walkers ceil(nw/4096)*6, nodes ceil(N/4096)*12 doubles
hipError_t launch_moments(int prec, const DomView* v, int dom, int64_t N, int64_t nw, const double* ref,
                          double* pw, double* pn, double* out, hipStream_t s);
hipError_t launch_advance(const DomView* views, int nd, uint32_t n, hipStream_t s);
// Two-way coupled particles of domain views[0] (dem_args: a device DemArgs,
// dem_impl.h): the particle update of step tstep + j, and the pose tables of
// step tstep from the particle state.
hipError_t launch_dem(const DomView* v, const void* dem_args, int32_t j, hipStream_t s);
hipError_t launch_dem_tables(const DomView* v, const void* dem_args, hipStream_t s);

// Scratch of the allocation-free moment read-out: a file-scope device array
// of kNoAllocDoubles doubles (1 MiB) in k_fp64.hip, one copy per GPU, held
// until the process ends.  noalloc_scratch returns its device address on the
// current device (looked up once per device and kept).
constexpr int64_t kNoAllocDoubles = 131072;
hipError_t noalloc_scratch(double** ptr);

// Scratch of the walker sort of one domain (device memory owned by the domain).
struct SortScratch {
  uint32_t* hist;  // 16 counters per bin (copy-major), bin totals, scan tile sums
  uint32_t* bin;   // [nw]
  uint32_t* rank;  // [nw]
  int32_t* cell;   // [nw]
  void* off;       // [3][nw] in the walker offset type
  int32_t* img;    // [3][nw]
  int32_t* wid;    // [nw]
  int64_t nbins;
};
// Regroup the walkers of domain `dom` of `views` by coarse mask block.
hipError_t launch_sort(int prec, const DomView* views, int dom, int64_t nw, const SortScratch& sc, hipStream_t s);
// Slot i holds walker i (after seeding).
hipError_t launch_ids_identity(const DomView* views, int dom, int64_t nw, hipStream_t s);
hipError_t launch_normals(uint64_t seed, uint32_t t, uint32_t purpose, int64_t n, double* z, hipStream_t s);

}  // namespace rwmi
