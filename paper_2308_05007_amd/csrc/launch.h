// Host-side launchers of the kernels (defined in k_fp64.hip and k_lowp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rwmi {
struct DomView;

// A multi-domain launch: `blocks` blocks over nd domains, boff (device) the
// block prefix per domain.
struct Work {
  const DomView* views;
  const int32_t* boff;
  int nd;
  int blocks;
  int flags;     // fluid kernel: kFlagXcd | kFlagNontemporal
  uint32_t k;    // step offset within the launch group
};
constexpr int kFlagXcd = 1;          // XCD-contiguous block order
constexpr int kFlagNontemporal = 2;  // non-temporal stores of f* and (u, rho)

hipError_t launch_prologue(const Work& w, hipStream_t s);
hipError_t launch_fluid_p64(int bs, const Work& w, hipStream_t s);
hipError_t launch_fluid_lowp(int prec, int bs, const Work& w, hipStream_t s);
hipError_t launch_walk_p64(int bs, const Work& w, hipStream_t s);
hipError_t launch_walk_lowp(int bs, const Work& w, hipStream_t s);
hipError_t launch_walk_slow_p64(int bs, const Work& w, hipStream_t s);
hipError_t launch_walk_slow_lowp(int bs, const Work& w, hipStream_t s);
hipError_t launch_init_p64(const DomView* v, int dom, int64_t N, const double u0[3], hipStream_t s);
hipError_t launch_init_lowp(int prec, const DomView* v, int dom, int64_t N, const double u0[3], hipStream_t s);
hipError_t launch_read_f_p64(const DomView* v, int dom, int64_t N, double* out, hipStream_t s);
hipError_t launch_read_f_lowp(int prec, const DomView* v, int dom, int64_t N, double* out, hipStream_t s);

// precision 0 is FP64 (rwmi::P64)
inline hipError_t launch_fluid(int prec, int bs, const Work& w, hipStream_t s) {
  return prec == 0 ? launch_fluid_p64(bs, w, s) : launch_fluid_lowp(prec, bs, w, s);
}
inline hipError_t launch_walk(int prec, int bs, const Work& w, hipStream_t s) {
  return prec == 0 ? launch_walk_p64(bs, w, s) : launch_walk_lowp(bs, w, s);
}
// one block per walker block (queue region), same block size as the walker kernel
inline hipError_t launch_walk_slow(int prec, int bs, const Work& w, hipStream_t s) {
  return prec == 0 ? launch_walk_slow_p64(bs, w, s) : launch_walk_slow_lowp(bs, w, s);
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
// partial buffers: walkers ceil(nw/4096)*6, nodes ceil(N/4096)*12 doubles
hipError_t launch_moments(int prec, const DomView* v, int dom, int64_t N, int64_t nw, const double* ref,
                          double* pw, double* pn, double* out, hipStream_t s);
hipError_t launch_advance(const DomView* views, int nd, uint32_t n, hipStream_t s);
hipError_t launch_normals(uint64_t seed, uint32_t t, uint32_t purpose, int64_t n, double* z, hipStream_t s);

}  // namespace rwmi
