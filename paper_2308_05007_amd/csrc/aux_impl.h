// Walker seeding, occupancy (Eq. 16) and the FP64 moment reductions.
#pragma once
#include "dev_common.h"
#include "lbm_impl.h"
#include "walk_impl.h"

namespace rwmi {

// Seeding at t = 0: walker w tries Philox blocks (w, 0xFFFFFFFF, 16 + a, 0).
// Writes cell, offsets (in the walker precision) and flag[w] = 1 if placed.
template <typename R>
__global__ void k_seed(const DomView* __restrict__ views, int dom, int kind, double cx, double cy, double cz,
                       double sigma, int band_axis, double band_lo, double band_hi, const double* __restrict__ xyz,
                       int64_t n, int attempts, int32_t* __restrict__ cell_out, R* __restrict__ off_out,
                       uint8_t* __restrict__ flag) {
  const DomView& V = views[dom];
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n) return;
  // particle centres at t = 0
  const double centre[3] = {cx, cy, cz};
  bool placed = false;
  int cell[3] = {0, 0, 0};
  double o[3] = {0, 0, 0};
  for (int at = 0; at < attempts && !placed; ++at) {
    double X[3];
    if (kind == 3) {
      X[0] = xyz[3 * w];
      X[1] = xyz[3 * w + 1];
      X[2] = xyz[3 * w + 2];
    } else {
      const U4 r = philox4x32_10((uint32_t)w, 0xFFFFFFFFu, 16u + (uint32_t)at, 0u, V.key0, V.key1);
      if (kind == 1) {
        double z0, z1, z2;
        gauss3(r, z0, z1, z2);
        X[0] = centre[0] + sigma * z0;
        X[1] = centre[1] + sigma * z1;
        X[2] = centre[2] + sigma * z2;
      } else {
        const uint32_t rr[3] = {r.x, r.y, r.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          double lo = V.bc[a] ? 1.0 : 0.0, hi = V.bc[a] ? (double)(V.n[a] - 1) : (double)V.n[a];
          if (kind == 2 && a == band_axis) {
            lo = band_lo;
            hi = band_hi;
          }
          X[a] = lo + unit_open(rr[a]) * (hi - lo);
        }
      }
    }
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double L = (double)V.n[a];
      double x = X[a];
      if (!V.bc[a]) {
        x = x - L * floor(x / L);
        if (x >= L) x = 0.0;
      } else if (x < 1.0 || x >= L - 1.0) {
        ok = false;
      }
      const double k = floor(x);
      cell[a] = (int)k;
      o[a] = (double)(R)(x - k);
    }
    if (!ok) continue;
    // inside a particle at t = 0?
    bool inside = false;
    for (int p = 0; p < V.np && !inside; ++p) {
      const DevParticle& P = V.parts[p];
      double pc[3], pv[3];
      particle_pose(P, 0, pc, pv);
      const double dx = axis_disp<double>(!V.bc[0], V.n[0], cell[0], pc[0], o[0]);
      const double dy = axis_disp<double>(!V.bc[1], V.n[1], cell[1], pc[1], o[1]);
      const double dz = axis_disp<double>(!V.bc[2], V.n[2], cell[2], pc[2], o[2]);
      if ((dx * dx + dy * dy) + dz * dz >= P.maskr * P.maskr) continue;
      // control points as given (seeding happens before the first step, at
      // the initial orientation)
      if (metaball_value<double>(gp(V.ctrl) + 4 * P.ctrl0, P.nc, dx, dy, dz) >= 1.0) inside = true;
    }
    if (inside) continue;
    placed = true;
  }
  flag[w] = placed ? 1 : 0;
  cell_out[w] = (int32_t)lin(V, cell[0], cell[1], cell[2]);
  off_out[w] = (R)o[0];
  off_out[n + w] = (R)o[1];
  off_out[2 * n + w] = (R)o[2];
}

// Scatter the placed walkers (exclusive prefix pos of flag) into the walker
// arrays, keeping their order.
template <typename R>
__global__ void k_seed_scatter(const DomView* __restrict__ views, int dom, int64_t n, const int32_t* __restrict__ cell_in,
                               const R* __restrict__ off_in, const uint8_t* __restrict__ flag,
                               const int32_t* __restrict__ pos, int64_t m) {
  const DomView& V = views[dom];
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n || !flag[w]) return;
  const int64_t k = pos[w];
  R* off = (R*)V.woff;
  V.wcell[k] = cell_in[w];
  off[k] = off_in[w];
  off[m + k] = off_in[n + w];
  off[2 * m + k] = off_in[2 * n + w];
  V.wimg[k] = 0;
  V.wimg[m + k] = 0;
  V.wimg[2 * m + k] = 0;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_occupancy(const DomView* __restrict__ views, int dom) {
  const DomView& V = views[dom];
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < V.nw)
    __hip_atomic_fetch_add(gp(V.occ) + gp(V.wcell)[w], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- profile
// Concentration profile along one axis (Eq. 16 summed over the two other
// axes): the number of walkers whose cell lies in each layer.  Exact integer
// counts in any order of addition.  Layers up to kProfileLds are counted in
// a block histogram in LDS first, then added to the global counts once per
// block and layer.
constexpr int kProfileLds = 4096;
constexpr int kProfileThreads = 256;
constexpr int kProfilePerThread = 16;

__global__ void __launch_bounds__(kProfileThreads) k_profile(const DomView* __restrict__ views, int dom, int axis,
                                                             uint32_t* __restrict__ counts) {
  __shared__ uint32_t h[kProfileLds];
  const DomView& V = views[dom];
  const int nl = V.n[axis];
  const bool lds = nl <= kProfileLds;
  if (lds)
    for (int i = threadIdx.x; i < nl; i += kProfileThreads) h[i] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kProfileThreads * kProfilePerThread;
  for (int k = 0; k < kProfilePerThread; ++k) {
    const int64_t w = base + (int64_t)k * kProfileThreads + threadIdx.x;
    if (w >= V.nw) break;
    const uint32_t c = (uint32_t)gp(V.wcell)[w];
    const uint32_t q1 = fdiv(c, V.dx);
    uint32_t layer;
    if (axis == 0) layer = c - q1 * (uint32_t)V.n[0];
    else if (axis == 1) layer = q1 - fdiv(q1, V.dy) * (uint32_t)V.n[1];
    else layer = fdiv(q1, V.dy);
    if (lds) __hip_atomic_fetch_add(&h[layer], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else __hip_atomic_fetch_add(gp(counts) + layer, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (lds)
    for (int i = threadIdx.x; i < nl; i += kProfileThreads)
      if (h[i]) __hip_atomic_fetch_add(gp(counts) + i, h[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- moments
// Deterministic FP64 reductions: chunk k covers elements [k*4096, (k+1)*4096);
// thread j of the 256-thread block adds elements j, j+256, ... in order, the
// block then folds the 256 partials by halving; the final kernel adds the
// chunk partials in chunk order.  The result does not depend on the launch
// configuration of the stepping kernels.
constexpr int kRedChunk = 4096;
constexpr int kRedThreads = 256;
constexpr int kWalkMom = 6;   // sum d[3], sum d^2[3]
constexpr int kNodeMom = 12;  // rho, rho u[3], (1-eps) u[3], (1-eps), eps us[3], eps

template <int K>
__device__ __forceinline__ void block_fold(double (*sh)[kRedThreads], double acc[K], double* out) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < K; ++k) sh[k][tid] = acc[k];
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int k = 0; k < K; ++k) sh[k][tid] = sh[k][tid] + sh[k][tid + h];
    }
    __syncthreads();
  }
  if (tid < K) out[tid] = sh[tid][0];
}

template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_mom_walkers(const DomView* __restrict__ views, int dom,
                                                             const double* __restrict__ ref, double* __restrict__ part) {
  __shared__ double sh[kWalkMom][kRedThreads];
  const DomView& V = views[dom];
  const R* off = (const R*)V.woff;
  const int64_t base = (int64_t)blockIdx.x * kRedChunk;
  double acc[kWalkMom] = {0, 0, 0, 0, 0, 0};
  const int nx = V.n[0], ny = V.n[1];
  for (int j = threadIdx.x; j < kRedChunk; j += kRedThreads) {
    const int64_t id = base + j;  // walker ids in order, whatever slot holds them
    if (id >= V.nw) break;
    const int64_t w = V.winv[id];
    const int32_t lc = V.wcell[w];
    const int c[3] = {lc % nx, (lc / nx) % ny, lc / (nx * ny)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t X = (int64_t)c[a] + (int64_t)V.wimg[a * V.nw + w] * (int64_t)V.n[a];
      const double dv = ((double)X - ref[a]) + (double)off[a * V.nw + w];
      acc[a] = acc[a] + dv;
      acc[3 + a] = acc[3 + a] + dv * dv;
    }
  }
  block_fold<kWalkMom>(sh, acc, part + (int64_t)blockIdx.x * kWalkMom);
}

template <typename U>
__global__ void __launch_bounds__(kRedThreads) k_mom_nodes(const DomView* __restrict__ views, int dom,
                                                           double* __restrict__ part) {
  __shared__ double sh[kNodeMom][kRedThreads];
  using C = typename Store<sizeof(U) == 8 ? P64 : P32>::C;
  __shared__ BlockParticles<C> sp;
  const DomView& V = views[dom];
  const int64_t base = (int64_t)blockIdx.x * kRedChunk;
  const int64_t last = (base + kRedChunk - 1 < V.N) ? base + kRedChunk - 1 : V.N - 1;
  const uint64_t done = V.tstep[0];  // steps completed
  const bool stepped = done > 0;
  // coupled particles: poses from the table the particle update wrote
  if (stepped && V.np > 0) cull_block<C>(V, (uint32_t)base, (uint32_t)last, done - 1, sp, V.dem_mask != 0ull);
  else if (threadIdx.x == 0) sp.cnt = 0;
  __syncthreads();
  double acc[kNodeMom];
#pragma unroll
  for (int k = 0; k < kNodeMom; ++k) acc[k] = 0.0;
  const U* uf = (const U*)V.u[stepped ? ((done - 1) & 1ull) : 0];
  const U* rf = (const U*)V.rho;
  const int nx = V.n[0], ny = V.n[1];
  for (int j = threadIdx.x; j < kRedChunk; j += kRedThreads) {
    const int64_t id = base + j;
    if (id >= V.N) break;
    const int nd[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((int64_t)nx * ny))};
    bool wall = false;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (V.bc[a] && (nd[a] == 0 || nd[a] == V.n[a] - 1)) wall = true;
    if (wall) continue;
    double es = 0.0, un[3] = {0.0, 0.0, 0.0};
    if (V.ibb) {
      // interpolated bounce-back: a node is solid or fluid; a solid node's
      // stored velocity is its particle's rigid velocity
      if (stepped && (V.smap[(done - 1) & 1ull][id] & kSolidBits)) {
        es = 1.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) un[a] = (double)uf[3 * id + a];
      }
    } else
    for (int k = 0; k < sp.cnt; ++k) {
      C dl[3];
      const double e = (double)node_eps<C>(V, sp, k, nd, dl);
      es = es + e;
      double up[3] = {sp.v[k][0], sp.v[k][1], sp.v[k][2]};
      if (((V.dem_mask >> sp.id[k]) & 1ull) && e > 0.0) {
        const double dd[3] = {(double)dl[0], (double)dl[1], (double)dl[2]};
        rigid_velocity<double>(sp.w[k], dd, up);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) un[a] = un[a] + e * up[a];
    }
    const double eps = es < 1.0 ? es : 1.0;
    const double r = (double)rf[id];
    acc[0] = acc[0] + r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double ua = (double)uf[3 * id + a];
      const double usa = es > 0.0 ? un[a] / es : 0.0;
      acc[1 + a] = acc[1 + a] + r * ua;
      acc[4 + a] = acc[4 + a] + (1.0 - eps) * ua;
      acc[8 + a] = acc[8 + a] + eps * usa;
    }
    acc[7] = acc[7] + (1.0 - eps);
    acc[11] = acc[11] + eps;
  }
  block_fold<kNodeMom>(sh, acc, part + (int64_t)blockIdx.x * kNodeMom);
}

// out: [0..5] walker sums, [6..17] node sums, [18..25] counters, [26] step
__global__ void k_mom_final(const DomView* __restrict__ views, int dom, const double* __restrict__ pw, int64_t nbw,
                            const double* __restrict__ pn, int64_t nbn, double* __restrict__ out) {
  const DomView& V = views[dom];
  const int tid = threadIdx.x;
  if (tid < kWalkMom) {
    double s = 0.0;
    for (int64_t b = 0; b < nbw; ++b) s = s + pw[b * kWalkMom + tid];
    out[tid] = s;
  } else if (tid < kWalkMom + kNodeMom) {
    const int k = tid - kWalkMom;
    double s = 0.0;
    for (int64_t b = 0; b < nbn; ++b) s = s + pn[b * kNodeMom + k];
    out[tid] = s;
  } else if (tid < kWalkMom + kNodeMom + kCounters) {
    const int k = tid - kWalkMom - kNodeMom;
    out[tid] = __longlong_as_double((long long)V.counters[k]);
  } else if (tid == kWalkMom + kNodeMom + kCounters) {
    out[tid] = __longlong_as_double((long long)V.tstep[0]);
  }
}

// End of a launch group: every domain of the launch has completed n more steps.
__global__ void k_advance(const DomView* __restrict__ views, int nd_count, uint32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nd_count) views[i].tstep[0] += n;
}

__global__ void k_normals(uint32_t k0, uint32_t k1, uint32_t t, uint32_t purpose, int64_t n, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const U4 r = philox4x32_10((uint32_t)i, t, purpose, 0u, k0, k1);
  double a, b, c;
  gauss3(r, a, b, c);
  z[3 * i] = a;
  z[3 * i + 1] = b;
  z[3 * i + 2] = c;
}

// ---------------------------------------------------------------- walker sort
// Walkers are kept grouped by coarse mask block (4^3 nodes) so that the
// walkers of a wavefront gather neighbouring velocities and share mask words.
// A counting sort: rank within the block's bin (wave-aggregated atomics, so
// the order inside a bin is arbitrary), exclusive scan of the bin counts,
// scatter to scratch, copy back.  Every result of the library is independent
// of the slot order (walker ids travel with the walkers; moments and
// read-back go by id), so the arbitrary order inside a bin changes nothing.

__device__ __forceinline__ uint32_t walker_bin(const DomView& V, int32_t cell) {
  const uint32_t lc = (uint32_t)cell;
  const uint32_t q1 = fdiv(lc, V.dx);
  const uint32_t z = fdiv(q1, V.dy);
  const uint32_t y = q1 - z * (uint32_t)V.n[1];
  const uint32_t x = lc - q1 * (uint32_t)V.n[0];
  return x / kMaskBlock + (uint32_t)V.mb[0] * (y / kMaskBlock + (uint32_t)V.mb[1] * (z / kMaskBlock));
}

// Every bin has kSortCopies counters, stored copy-major (counter copy * nbins
// + bin, so the copies of a bin sit in different cache lines); a block uses
// copy blockIdx mod kSortCopies, so that the walkers of a dense bin do not
// all queue on one address.  The starts are then taken bin by bin: bin totals,
// exclusive scan over the bins, then the copies of each bin in order.
constexpr int kSortCopies = 16;

// bin[w] (its counter) and rank[w] (position among the walkers of that
// counter); hist[counter] ends as the count.
__global__ void k_sort_rank(const DomView* __restrict__ views, int dom, uint32_t* __restrict__ hist,
                            uint32_t* __restrict__ bin, uint32_t* __restrict__ rank) {
  const DomView& V = views[dom];
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = w < V.nw;
  const uint32_t nbins = (uint32_t)V.mb[0] * (uint32_t)V.mb[1] * (uint32_t)V.mb[2];
  const uint32_t key = active ? (uint32_t)(blockIdx.x % kSortCopies) * nbins + walker_bin(V, gp(V.wcell)[w]) : 0u;
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(active);
  uint32_t r = 0;
  while (todo) {
    // the lowest pending lane's key: one atomic for all lanes holding it
    const int leader = __ffsll((long long)todo) - 1;
    const uint32_t k = __shfl(key, leader);
    const unsigned long long same = __ballot(active && key == k) & todo;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&hist[k], (uint32_t)__popcll(same));
    base = __shfl(base, leader);
    if ((same >> lane) & 1ull) r = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  if (active) {
    gp(bin)[w] = key;
    gp(rank)[w] = r;
  }
}

// Exclusive scan of n counts in place: tiles of kScanTile counts scanned by
// one block each (every thread a contiguous run of 4, loaded and stored
// coalesced), the tile sums scanned by one block, then added to the tiles.
constexpr int kScanThreads = 1024;
constexpr int kScanTile = 4 * kScanThreads;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s, uint32_t& total) {
  const int tid = threadIdx.x;
  s[tid] = v;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {  // Hillis-Steele inclusive scan
    const uint32_t u = tid >= o ? s[tid - o] : 0u;
    __syncthreads();
    s[tid] += u;
    __syncthreads();
  }
  total = s[kScanThreads - 1];
  return s[tid] - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(uint32_t* __restrict__ a, int64_t n,
                                                             uint32_t* __restrict__ tsum) {
  __shared__ uint32_t s[kScanThreads];
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  const auto g = gp(a);
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = i0 + k < n ? g[i0 + k] : 0u;
  uint32_t total;
  uint32_t run = block_exclusive_scan((v[0] + v[1]) + (v[2] + v[3]), s, total);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i0 + k < n) g[i0 + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) gp(tsum)[blockIdx.x] = total;
}

// Exclusive scan of m <= kScanThreads * 64 tile sums, one block.
__global__ void __launch_bounds__(kScanThreads) k_scan_sums(uint32_t* __restrict__ t, int64_t m) {
  __shared__ uint32_t s[kScanThreads];
  const int64_t per = (m + kScanThreads - 1) / kScanThreads;
  const int64_t b = threadIdx.x * per, e = (b + per < m) ? b + per : m;
  uint32_t sum = 0;
  for (int64_t i = b; i < e; ++i) sum += t[i];
  uint32_t total;
  uint32_t run = block_exclusive_scan(sum, s, total);
  for (int64_t i = b; i < e; ++i) {
    const uint32_t c = t[i];
    t[i] = run;
    run += c;
  }
}

__global__ void k_scan_add(uint32_t* __restrict__ a, int64_t n, const uint32_t* __restrict__ tsum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) gp(a)[i] += gp(tsum)[i / kScanTile];
}

// total[b] = sum over the copies of bin b.
__global__ void k_bin_totals(const uint32_t* __restrict__ cnt, int64_t nbins, uint32_t* __restrict__ total) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < kSortCopies; ++c) s += gp(cnt)[c * nbins + b];
  gp(total)[b] = s;
}

// Counts of the copies of bin b become their starts, from the bin's start.
__global__ void k_bin_starts(uint32_t* __restrict__ cnt, int64_t nbins, const uint32_t* __restrict__ start) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  uint32_t run = gp(start)[b];
#pragma unroll
  for (int c = 0; c < kSortCopies; ++c) {
    const uint32_t k = gp(cnt)[c * nbins + b];
    gp(cnt)[c * nbins + b] = run;
    run += k;
  }
}

// Scatter every walker to slot start[bin] + rank in the scratch arrays.
template <typename R>
__global__ void k_sort_scatter(const DomView* __restrict__ views, int dom, const uint32_t* __restrict__ start,
                               const uint32_t* __restrict__ bin, const uint32_t* __restrict__ rank,
                               int32_t* __restrict__ cell2, R* __restrict__ off2, int32_t* __restrict__ img2,
                               int32_t* __restrict__ wid2) {
  const DomView& V = views[dom];
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= V.nw) return;
  const int64_t nw = V.nw;
  const int64_t d = (int64_t)gp(start)[gp(bin)[w]] + gp(rank)[w];
  gp(cell2)[d] = gp(V.wcell)[w];
  gp(wid2)[d] = gp(V.wid)[w];
  const auto off = gp((const R*)V.woff);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gp(off2)[a * nw + d] = off[a * nw + w];
    gp(img2)[a * nw + d] = gp(V.wimg)[a * nw + w];
  }
}

// Copy the sorted scratch back.
template <typename R>
__global__ void k_sort_back(const DomView* __restrict__ views, int dom, const int32_t* __restrict__ cell2,
                            const R* __restrict__ off2, const int32_t* __restrict__ img2,
                            const int32_t* __restrict__ wid2) {
  const DomView& V = views[dom];
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= V.nw) return;
  const int64_t nw = V.nw;
  gp(V.wcell)[w] = gp(cell2)[w];
  gp(V.wid)[w] = gp(wid2)[w];
  const auto off = gp((R*)V.woff);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    off[a * nw + w] = gp(off2)[a * nw + w];
    gp(V.wimg)[a * nw + w] = gp(img2)[a * nw + w];
  }
}

// Slot i holds walker i (after seeding).
__global__ void k_ids_identity(const DomView* __restrict__ views, int dom) {
  const DomView& V = views[dom];
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= V.nw) return;
  gp(V.wid)[w] = (int32_t)w;
}

// The id -> slot map, built when a read-out needs walkers in id order.
__global__ void k_ids_inverse(const DomView* __restrict__ views, int dom) {
  const DomView& V = views[dom];
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= V.nw) return;
  gp(V.winv)[gp(V.wid)[w]] = (int32_t)w;
}

}  // namespace rwmi
