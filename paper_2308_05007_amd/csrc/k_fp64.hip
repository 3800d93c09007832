// FP64 kernels (compiled with -ffp-contract=off: every double operation is
// a separately rounded IEEE operation) and the precision-independent ones.
#include <mutex>

#include "aux_impl.h"
#include "dem_impl.h"
#include "launch.h"
#include "step_impl.h"

// Moment partials, staging output and reference point of the allocation-free
// moment read-out.  In host code this name is only a stand-in for the symbol:
// kernels get the address noalloc_scratch looked up on their device.
static __device__ __align__(256) double scratch[rwmi::kNoAllocDoubles];

namespace rwmi {

hipError_t noalloc_scratch(double** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (double*)p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_ibb_links_p64(const DomView* v, int dom, int32_t j, bool dem, unsigned blocks, hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  blocks = kLinkGrid;  // the pass strides over the listed nodes
  if (dem) k_ibb_links<P64, true><<<blocks, 256, 0, s>>>(v, dom, j);
  else k_ibb_links<P64, false><<<blocks, 256, 0, s>>>(v, dom, j);
  return hipGetLastError();
}

hipError_t launch_step_p64(int bs, const StepArgs& a, hipStream_t s) {
  const unsigned g = (unsigned)step_grid(a.nb, (a.flags & kFlagXcd) != 0);
  if (g == 0) return hipSuccess;
  if (a.flags & kFlagIbb) {  // bounce-back coupling: two lattices, 256 threads per block; the link
                             // pass carries the coupled particles' momentum exchange
    k_step<P64, 256, false, false, true><<<g, 256, 0, s>>>(a, a.views, a.boff);
    return hipGetLastError();
  }
  if (a.flags & kFlagDem) {  // coupled particles: 256 threads per block
    if (a.inplace) k_step<P64, 256, true, true><<<g, 256, 0, s>>>(a, a.views, a.boff);
    else k_step<P64, 256, false, true><<<g, 256, 0, s>>>(a, a.views, a.boff);
    return hipGetLastError();
  }
  if (a.inplace) {
    switch (bs) {
      case 128: k_step<P64, 128, true><<<g, 128, 0, s>>>(a, a.views, a.boff); break;
      case 512: k_step<P64, 512, true><<<g, 512, 0, s>>>(a, a.views, a.boff); break;
      default: k_step<P64, 256, true><<<g, 256, 0, s>>>(a, a.views, a.boff); break;
    }
  } else {
    switch (bs) {
      case 128: k_step<P64, 128, false><<<g, 128, 0, s>>>(a, a.views, a.boff); break;
      case 512: k_step<P64, 512, false><<<g, 512, 0, s>>>(a, a.views, a.boff); break;
      default: k_step<P64, 256, false><<<g, 256, 0, s>>>(a, a.views, a.boff); break;
    }
  }
  return hipGetLastError();
}

// The particle update of step tstep + j of domain views[0]: one block of 64
// threads (one per particle).
__global__ void __launch_bounds__(2 * kMaxParticles) k_dem(const DomView* __restrict__ views,
                                                          const DemArgs* __restrict__ da,
                                            int32_t j) {
  __shared__ DemLds S;
  const DomView& V = views[0];
  const DemArgs A = *da;  // parameters in registers for the whole update
  dem_block(V, A, step_of(V, j), S);
}

__global__ void __launch_bounds__(64) k_dem_tables(const DomView* __restrict__ views, const DemArgs* __restrict__ da) {
  const DomView& V = views[0];
  dem_tables(V, *da, step_of(V, 0));
}

hipError_t launch_dem(const DomView* v, const void* dem_args, int32_t j, hipStream_t s) {
  k_dem<<<1, 2 * kMaxParticles, 0, s>>>(v, (const DemArgs*)dem_args, j);
  return hipGetLastError();
}

hipError_t launch_dem_tables(const DomView* v, const void* dem_args, hipStream_t s) {
  k_dem_tables<<<1, 64, 0, s>>>(v, (const DemArgs*)dem_args);
  return hipGetLastError();
}

hipError_t launch_init_p64(const DomView* v, int dom, int64_t N, const double u0[3], hipStream_t s) {
  k_init<P64><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(v, dom, u0[0], u0[1], u0[2]);
  return hipGetLastError();
}

hipError_t launch_read_f_p64(const DomView* v, int dom, int64_t N, double* out, hipStream_t s) {
  k_read_f<P64><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(v, dom, out);
  return hipGetLastError();
}

hipError_t launch_seed(int prec, const DomView* v, int dom, int kind, const double c[3], double sigma, int axis,
                       double lo, double hi, const double* xyz, int64_t n, int attempts, int32_t* cell, void* off,
                       uint8_t* flag, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  if (prec == P64)
    k_seed<double><<<g, 256, 0, s>>>(v, dom, kind, c[0], c[1], c[2], sigma, axis, lo, hi, xyz, n, attempts, cell,
                                     (double*)off, flag);
  else
    k_seed<float><<<g, 256, 0, s>>>(v, dom, kind, c[0], c[1], c[2], sigma, axis, lo, hi, xyz, n, attempts, cell,
                                    (float*)off, flag);
  return hipGetLastError();
}

hipError_t launch_seed_scatter(int prec, const DomView* v, int dom, int64_t n, const int32_t* cell, const void* off,
                               const uint8_t* flag, const int32_t* pos, int64_t m, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  if (prec == P64)
    k_seed_scatter<double><<<g, 256, 0, s>>>(v, dom, n, cell, (const double*)off, flag, pos, m);
  else
    k_seed_scatter<float><<<g, 256, 0, s>>>(v, dom, n, cell, (const float*)off, flag, pos, m);
  return hipGetLastError();
}

hipError_t launch_occupancy(const DomView* v, int dom, uint32_t* occ, int64_t N, int64_t nw, hipStream_t s) {
  k_fill_u32<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(occ, N, 0u);
  if (nw > 0) k_occupancy<<<(unsigned)((nw + 255) / 256), 256, 0, s>>>(v, dom);
  return hipGetLastError();
}

hipError_t launch_profile(const DomView* v, int dom, int axis, int n_layers, int64_t nw, uint32_t* counts,
                          hipStream_t s) {
  k_fill_u32<<<(unsigned)((n_layers + 255) / 256), 256, 0, s>>>(counts, n_layers, 0u);
  if (nw > 0) {
    const int64_t per = (int64_t)kProfileThreads * kProfilePerThread;
    k_profile<<<(unsigned)((nw + per - 1) / per), kProfileThreads, 0, s>>>(v, dom, axis, counts);
  }
  return hipGetLastError();
}

hipError_t launch_moments(int prec, const DomView* v, int dom, int64_t N, int64_t nw, const double* ref, double* pw,
                          double* pn, double* out, hipStream_t s) {
  const int64_t nbw = (nw + kRedChunk - 1) / kRedChunk;
  const int64_t nbn = (N + kRedChunk - 1) / kRedChunk;
  if (nbw > 0) {
    k_ids_inverse<<<(unsigned)((nw + 255) / 256), 256, 0, s>>>(v, dom);
    if (prec == P64) k_mom_walkers<double><<<(unsigned)nbw, kRedThreads, 0, s>>>(v, dom, ref, pw);
    else k_mom_walkers<float><<<(unsigned)nbw, kRedThreads, 0, s>>>(v, dom, ref, pw);
  }
  if (prec == P64) k_mom_nodes<double><<<(unsigned)nbn, kRedThreads, 0, s>>>(v, dom, pn);
  else k_mom_nodes<float><<<(unsigned)nbn, kRedThreads, 0, s>>>(v, dom, pn);
  k_mom_final<<<1, 64, 0, s>>>(v, dom, pw, nbw, pn, nbn, out);
  return hipGetLastError();
}

hipError_t launch_sort(int prec, const DomView* views, int dom, int64_t nw, const SortScratch& sc, hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  const unsigned gw = (unsigned)((nw + 255) / 256);
  // hist: counters [kSortCopies][nbins], bin totals [nbins], scan tile sums
  const int64_t nb = sc.nbins, nc = nb * kSortCopies;
  uint32_t* total = sc.hist + nc;
  uint32_t* tsum = total + nb;
  const unsigned gb = (unsigned)((nb + 255) / 256);
  const int64_t tiles = (nb + kScanTile - 1) / kScanTile;
  k_fill_u32<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>(sc.hist, nc, 0u);
  k_sort_rank<<<gw, 256, 0, s>>>(views, dom, sc.hist, sc.bin, sc.rank);
  k_bin_totals<<<gb, 256, 0, s>>>(sc.hist, nb, total);
  k_scan_tiles<<<(unsigned)tiles, kScanThreads, 0, s>>>(total, nb, tsum);
  k_scan_sums<<<1, kScanThreads, 0, s>>>(tsum, tiles);
  k_scan_add<<<gb, 256, 0, s>>>(total, nb, tsum);
  k_bin_starts<<<gb, 256, 0, s>>>(sc.hist, nb, total);
  if (prec == P64) {
    k_sort_scatter<double><<<gw, 256, 0, s>>>(views, dom, sc.hist, sc.bin, sc.rank, sc.cell, (double*)sc.off, sc.img,
                                               sc.wid);
    k_sort_back<double><<<gw, 256, 0, s>>>(views, dom, sc.cell, (const double*)sc.off, sc.img, sc.wid);
  } else {
    k_sort_scatter<float><<<gw, 256, 0, s>>>(views, dom, sc.hist, sc.bin, sc.rank, sc.cell, (float*)sc.off, sc.img,
                                              sc.wid);
    k_sort_back<float><<<gw, 256, 0, s>>>(views, dom, sc.cell, (const float*)sc.off, sc.img, sc.wid);
  }
  return hipGetLastError();
}

hipError_t launch_ids_identity(const DomView* views, int dom, int64_t nw, hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  k_ids_identity<<<(unsigned)((nw + 255) / 256), 256, 0, s>>>(views, dom);
  return hipGetLastError();
}

hipError_t launch_advance(const DomView* views, int nd, uint32_t n, hipStream_t s) {
  k_advance<<<(nd + 63) / 64, 64, 0, s>>>(views, nd, n);
  return hipGetLastError();
}

hipError_t launch_normals(uint64_t seed, uint32_t t, uint32_t purpose, int64_t n, double* z, hipStream_t s) {
  k_normals<<<(unsigned)((n + 255) / 256), 256, 0, s>>>((uint32_t)seed, (uint32_t)(seed >> 32), t, purpose, n, z);
  return hipGetLastError();
}

}  // namespace rwmi
