// Random walkers (Eq. 2) on the lattice velocity field, one block function
// run by the walker blocks of the fused step launch.
//
// Fast path (one thread per walker slot): trilinear interpolation of u(t)
// between node centres (x, then y, then z), three normals from the Philox
// block (id, t, 0, 0) of the walker id the slot holds, step
// dl = u + z sqrt(2D).  The coarse cull mask of the particles at t+1 gives
// the candidates at the start cell (its dilated block covers the end of a
// short step) and, for a long step, at the end cell; float bounding-sphere
// tests on the prologue's sphere table filter them.  A walker with no
// candidate particle at either end can be neither type II nor IV (Sec.
// 2.4.2), so it is moved here (walls, renormalisation).  Walkers with a
// candidate are compacted into the block's LDS queue with a wavefront ballot.
//
// Near-surface path (the queued walkers, packed into the first waves of the
// same block): the full classification against the particles at t+1 (types
// I-IV), Algorithm 1 and Algorithm 2 for type IV, the refill of type II, then
// walls and renormalisation.
#pragma once
#include "dev_common.h"

namespace rwmi {

template <typename R> __device__ __forceinline__ R prev_value(R x);
template <> __device__ __forceinline__ double prev_value<double>(double x) {
  return __longlong_as_double(__double_as_longlong(x) - 1);  // x > 0
}
template <> __device__ __forceinline__ float prev_value<float>(float x) {
  return __int_as_float(__float_as_int(x) - 1);
}

__device__ __forceinline__ int64_t lin(const DomView& V, int x, int y, int z) {
  return (int64_t)x + (int64_t)V.n[0] * ((int64_t)y + (int64_t)V.n[1] * z);
}

// Coarse mask block of the cell that contains cell c + offset x (x need not be
// in [0,1)); periodic wrap, clamped at wall axes (the boundary blocks of the
// mask extend to infinity there).
template <typename R>
__device__ __forceinline__ int64_t mask_index(const DomView& V, const int c[3], const R x[3]) {
  int b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int k = c[a] + (int)floor(x[a]);
    const int n = V.n[a];
    if (!V.bc[a]) {
      if (k < 0 || k >= n) {
        k %= n;
        if (k < 0) k += n;
      }
    } else {
      k = k < 0 ? 0 : (k >= n ? n - 1 : k);
    }
    b[a] = k / kMaskBlock;
  }
  return b[0] + V.mb[0] * (b[1] + V.mb[1] * b[2]);
}

// Particle pose at t+1 from the pose table of step t.
__device__ __forceinline__ gconst<double> pose_next(const DomView& V, int ps, int p) {
  return gp((const double*)V.pose[ps]) + kPoseRec * (V.np + p);
}

template <typename R>
__device__ __forceinline__ R particle_M_at(const DomView& V, int ps, int p, const int c[3], const R x[3]) {
  const auto pc = pose_next(V, ps, p);
  const R dx = axis_disp<R>(!V.bc[0], V.n[0], c[0], pc[0], x[0]);
  const R dy = axis_disp<R>(!V.bc[1], V.n[1], c[1], pc[1], x[1]);
  const R dz = axis_disp<R>(!V.bc[2], V.n[2], c[2], pc[2], x[2]);
  const auto P = gp(V.parts) + p;
  return metaball_value<R>(gp(ctrl_of<R>(V, next_slot(ps))) + 4 * P->ctrl0, P->nc, dx, dy, dz);
}

template <typename R>
__device__ __forceinline__ void particle_grad_at(const DomView& V, int ps, int p, const int c[3], const R x[3], R g[3]) {
  const auto pc = pose_next(V, ps, p);
  const R dx = axis_disp<R>(!V.bc[0], V.n[0], c[0], pc[0], x[0]);
  const R dy = axis_disp<R>(!V.bc[1], V.n[1], c[1], pc[1], x[1]);
  const R dz = axis_disp<R>(!V.bc[2], V.n[2], c[2], pc[2], x[2]);
  const auto P = gp(V.parts) + p;
  metaball_grad<R>(gp(ctrl_of<R>(V, next_slot(ps))) + 4 * P->ctrl0, P->nc, dx, dy, dz, g);
}

// Is (c + x) within the sphere (c_p(t+1), rb_p + 1/2) of particle p, enlarged
// by kSphereMargin?  A float test on the sphere table the prologue wrote for
// step t; the margin covers the float rounding, so every point of the exact
// sphere passes.  A walker it passes goes to the exact near-surface path.
template <typename R>
__device__ __forceinline__ bool near_sphere(const DomView& V, int ps, int p, const int c[3], const R x[3]) {
  using F4 = float __attribute__((ext_vector_type(4)));
  const F4 sp = gp((const F4*)V.sph[ps])[p];
  const float sc[3] = {sp.x, sp.y, sp.z};
  float d2 = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float d = ((float)c[a] + (float)x[a]) - sc[a];
    if (!V.bc[a]) {
      const float L = (float)V.n[a];
      d = d - L * rintf(d * (1.0f / L));
    }
    d2 += d * d;
  }
  return d2 < sp.w;
}

template <typename R>
__device__ __forceinline__ unsigned long long mask_at(const DomView& V, int ps, const int c[3], const R x[3]) {
  return gp((const unsigned long long*)V.mask[ps])[mask_index<R>(V, c, x)];
}

// Coarse mask word of the cell c itself (c inside the lattice).
__device__ __forceinline__ unsigned long long mask_at_cell(const DomView& V, int ps, const int c[3]) {
  static_assert(kMaskBlock == 4, "coarse block index by shift");
  const uint32_t i = ((uint32_t)c[0] >> 2) +
                     (uint32_t)V.mb[0] * (((uint32_t)c[1] >> 2) + (uint32_t)V.mb[1] * ((uint32_t)c[2] >> 2));
  return gp((const unsigned long long*)V.mask[ps])[i];
}

// Lowest index of a particle whose own M >= 1 at (c + x), or -1.  Particles
// whose bounding sphere (rb + 1/2) is farther than the point are skipped: M < 1
// there (bounding-radius lemma), so the result is that of testing all.
template <typename R>
__device__ __forceinline__ int inside_any(const DomView& V, int ps, const int c[3], const R x[3]) {
  // only the particles whose mask bit is set for the point's coarse block can
  // contain it; visit them in ascending index order
  unsigned long long bits = mask_at<R>(V, ps, c, x);
  while (bits) {
    const int p = __ffsll((long long)bits) - 1;
    bits &= bits - 1ull;
    const auto pc = pose_next(V, ps, p);
    const R dx = axis_disp<R>(!V.bc[0], V.n[0], c[0], pc[0], x[0]);
    const R dy = axis_disp<R>(!V.bc[1], V.n[1], c[1], pc[1], x[1]);
    const R dz = axis_disp<R>(!V.bc[2], V.n[2], c[2], pc[2], x[2]);
    const auto P = gp(V.parts) + p;
    const R r2 = (dx * dx + dy * dy) + dz * dz;
    const double mr = P->maskr;
    if (r2 >= (R)(mr * mr)) continue;
    if (metaball_value<R>(gp(ctrl_of<R>(V, next_slot(ps))) + 4 * P->ctrl0, P->nc, dx, dy, dz) >= (R)1) return p;
  }
  return -1;
}

// Algorithm 1 on x(s) = a0 + s dir between s_out (M < 1) and s_in (M >= 1):
// midpoint in s, converged when |M - 1| < 1e-3, at most imax evaluations.
template <typename R>
__device__ __forceinline__ bool bisect(const DomView& V, int ps, int p, const int c[3], const R a0[3], const R dir[3],
                                       R s_out, R s_in, int imax, R& s_res) {
  for (int it = 1; it <= imax; ++it) {
    const R sm = (R)0.5 * (s_out + s_in);
    const R x[3] = {a0[0] + sm * dir[0], a0[1] + sm * dir[1], a0[2] + sm * dir[2]};
    const R m = particle_M_at<R>(V, ps, p, c, x);
    if (fabs(m - (R)1) < (R)1e-3) {
      s_res = sm;
      return true;
    }
    if (m < (R)1) s_out = sm;
    else s_in = sm;
  }
  return false;
}

// Wall reflection on wall axes (halfway planes at 1 and n-1, one reflection
// per axis).  Returns true if any coordinate was reflected.
template <typename R>
__device__ __forceinline__ bool reflect_walls(const DomView& V, const int c[3], R xn[3]) {
  bool refl = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!V.bc[a]) continue;
    const R lo = (R)(1.0 - (double)c[a]);
    const R hi = (R)((double)(V.n[a] - 1) - (double)c[a]);
    if (xn[a] < lo) {
      xn[a] = (R)2 * lo - xn[a];
      refl = true;
    } else if (xn[a] >= hi) {
      xn[a] = (R)2 * hi - xn[a];
      if (xn[a] == hi) xn[a] = prev_value<R>(hi);
      refl = true;
    }
  }
  return refl;
}

template <typename R>
__device__ __forceinline__ bool outside_walls(const DomView& V, const int c[3], const R xn[3]) {
  bool out = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!V.bc[a]) continue;
    const R lo = (R)(1.0 - (double)c[a]);
    const R hi = (R)((double)(V.n[a] - 1) - (double)c[a]);
    if (xn[a] < lo || xn[a] >= hi) out = true;
  }
  return out;
}

template <typename R>
__device__ __forceinline__ bool finite3(const R x[3]) {
  return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// Write back (cell, offset in [0,1), image counts on periodic wrap).
template <typename R>
__device__ __forceinline__ void store_walker(const DomView& V, int64_t w, int c[3], const R xn[3]) {
  const auto off = gp((R*)V.woff);
  const auto img = gp(V.wimg);
  const int64_t nw = V.nw;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R k = floor(xn[a]);
    R of = xn[a] - k;
    if (of == (R)1) {
      of = (R)0;
      k = k + (R)1;
    }
    int cc = c[a] + (int)k;
    if (!V.bc[a]) {
      const int n = V.n[a];
      if (cc < 0 || cc >= n) {
        const int q = cc >= 0 ? cc / n : -((-cc + n - 1) / n);  // floor(cc / n)
        cc -= q * n;
        img[a * nw + w] += q;
      }
    }
    c[a] = cc;
    off[a * nw + w] = of;
  }
  gp(V.wcell)[w] = (int32_t)((uint32_t)c[0] + (uint32_t)V.n[0] * ((uint32_t)c[1] + (uint32_t)V.n[1] * (uint32_t)c[2]));
}

// LDS of a walker block: the near-surface queue of its own walkers.
template <typename R, int BS>
struct WalkLds {
  uint32_t s_q[BS / 64], s_r[BS / 64];
  int32_t id[BS];
  R dl[3][BS];
};

template <int P>
__device__ void walk_near_surface(const DomView& V, uint64_t t, int64_t w, const typename Store<P>::O dl[3]);

// Walkers [lblock BS, (lblock + 1) BS) of a domain through step t.  Every
// thread of the block calls it.
template <int P, int BS>
__device__ __forceinline__ void walk_block(const DomView& V, int64_t lblock, uint64_t t,
                                           WalkLds<typename Store<P>::O, BS>& L) {
  using R = typename Store<P>::O;
  using U = typename Store<P>::U;
  const int64_t w = lblock * BS + threadIdx.x;
  const bool active = w < V.nw;
  const int ps = pose_slot(t);  // pose table and cull mask of step t
  bool queue = false;
  bool refl = false;
  R dl[3] = {(R)0, (R)0, (R)0};
  int c[3] = {0, 0, 0};
  R o[3] = {(R)0, (R)0, (R)0}, xf[3] = {(R)0, (R)0, (R)0};
  unsigned long long bits0 = 0ull;
  if (active) {
    const int par = (int)(t & 1ull);  // velocity buffer of step t
    const int nx = V.n[0], ny = V.n[1];
    const uint32_t lc = (uint32_t)gp(V.wcell)[w];
    const uint32_t q1 = fdiv(lc, V.dx);
    const int cz = (int)fdiv(q1, V.dy);
    c[0] = (int)(lc - q1 * (uint32_t)nx);
    c[1] = (int)q1 - cz * ny;
    c[2] = cz;
    const auto off = gp((const R*)V.woff);
    o[0] = off[w];
    o[1] = off[V.nw + w];
    o[2] = off[2 * V.nw + w];
    // trilinear interpolation between node centres
    int b0[3], b1[3];
    R wt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int b;
      if (o[a] >= (R)0.5) {
        b = c[a];
        wt[a] = o[a] - (R)0.5;
      } else {
        b = c[a] - 1;
        wt[a] = o[a] + (R)0.5;
      }
      int b1a = b + 1;
      if (b < 0) b += V.n[a];
      if (b1a >= V.n[a]) b1a -= V.n[a];
      b0[a] = b;
      b1[a] = b1a;
    }
    // one load per corner: (ux, uy, uz) of a node is 3 consecutive U, which
    // the compiler merges into one access.  All eight are issued, with the
    // cull-mask word of the start cell, before the normals are drawn, so that
    // the Philox rounds run while they are in flight.
    const auto uf = gp((const U*)V.u[par]);
    // node indices in 32 bits (fewer than 2^31 nodes): corner (0,0,0) plus
    // per-axis steps to the upper corner, which wrap on periodic axes
    const uint32_t unx = (uint32_t)nx, unxy = unx * (uint32_t)ny;
    const uint32_t i000 = (uint32_t)b0[0] + unx * ((uint32_t)b0[1] + (uint32_t)ny * (uint32_t)b0[2]);
    const uint32_t sx = (uint32_t)(b1[0] - b0[0]), sy = (uint32_t)(b1[1] - b0[1]) * unx,
                   sz = (uint32_t)(b1[2] - b0[2]) * unxy;
    U cu[2][2][2][3];
#pragma unroll
    for (int zz = 0; zz < 2; ++zz)
#pragma unroll
      for (int yy = 0; yy < 2; ++yy) {
        const uint32_t i0 = i000 + (yy ? sy : 0u) + (zz ? sz : 0u);
        const auto lo = uf + 3ull * i0, hi = uf + 3ull * (i0 + sx);
#pragma unroll
        for (int cpt = 0; cpt < 3; ++cpt) {
          cu[zz][yy][0][cpt] = lo[cpt];
          cu[zz][yy][1][cpt] = hi[cpt];
        }
      }
    if (V.np > 0) bits0 = mask_at_cell(V, ps, c);
    // Brownian step (Eq. 2 with dt = 1): normals of the walker id's Philox block
    const U4 r = philox4x32_10((uint32_t)gp(V.wid)[w], (uint32_t)t, 0u, 0u, V.key0, V.key1);
    R zn[3];
    if constexpr (P == P64) {
      double z0, z1, z2;
      gauss3(r, z0, z1, z2);
      zn[0] = z0 * V.sD;
      zn[1] = z1 * V.sD;
      zn[2] = z2 * V.sD;
    } else {
      float z0, z1, z2;
      gauss3_fast(r, z0, z1, z2);
      zn[0] = z0 * V.sD_f;
      zn[1] = z1 * V.sD_f;
      zn[2] = z2 * V.sD_f;
    }
    // trilinear interpolation of u(t): x, then y, then z
    R Ui[3];
    {
      R v[2][2][3];
#pragma unroll
      for (int zz = 0; zz < 2; ++zz)
#pragma unroll
        for (int yy = 0; yy < 2; ++yy) {
#pragma unroll
          for (int cpt = 0; cpt < 3; ++cpt)
            v[zz][yy][cpt] = ((R)1 - wt[0]) * (R)cu[zz][yy][0][cpt] + wt[0] * (R)cu[zz][yy][1][cpt];
        }
#pragma unroll
      for (int cpt = 0; cpt < 3; ++cpt) {
        const R v0 = ((R)1 - wt[1]) * v[0][0][cpt] + wt[1] * v[0][1][cpt];
        const R v1 = ((R)1 - wt[1]) * v[1][0][cpt] + wt[1] * v[1][1][cpt];
        Ui[cpt] = ((R)1 - wt[2]) * v0 + wt[2] * v1;
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) dl[a] = Ui[a] + zn[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) xf[a] = o[a] + dl[a];
    if (V.np > 0) {
      // a walker that starts and ends outside every bounding sphere is
      // neither type II nor IV (M < 1 outside rb); candidates come from the
      // coarse mask (the start word covers the end of a short step), the
      // sphere filter decides
      unsigned long long bits = bits0;
      if (!(fabs(dl[0]) <= (R)kMaskReach && fabs(dl[1]) <= (R)kMaskReach && fabs(dl[2]) <= (R)kMaskReach))
        bits |= mask_at<R>(V, ps, c, xf);
      while (bits && !queue) {
        const int p = __ffsll((long long)bits) - 1;
        bits &= bits - 1ull;
        queue = near_sphere<R>(V, ps, p, c, o) || near_sphere<R>(V, ps, p, c, xf);
      }
    }
    if (!queue) {
      R xn[3] = {xf[0], xf[1], xf[2]};
      if (!finite3<R>(xn)) {
        counter_add(&V.counters[kReturned], 1ull);
#pragma unroll
        for (int a = 0; a < 3; ++a) xn[a] = o[a];
      } else {
        refl = reflect_walls<R>(V, c, xn);
        if (refl) {
          if (outside_walls<R>(V, c, xn)) {
            counter_add(&V.counters[kReturned], 1ull);
#pragma unroll
            for (int a = 0; a < 3; ++a) xn[a] = o[a];
          } else if (V.np > 0) {
            unsigned long long bits = mask_at<R>(V, ps, c, xn);
            while (bits && !queue) {
              const int p = __ffsll((long long)bits) - 1;
              bits &= bits - 1ull;
              queue = near_sphere<R>(V, ps, p, c, xn);  // the reflected point may be inside a particle
            }
            if (queue) refl = false;
          }
        }
      }
      if (!queue) store_walker<R>(V, w, c, xn);
    }
  }
  // wavefront-ballot compaction of the near-surface walkers into the block's
  // LDS queue: ballot and popcount per wave, prefix over the waves
  constexpr int kWaves = BS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long qm = __ballot(queue);
  const unsigned long long rm = __ballot(refl);
  if (lane == 0) {
    L.s_q[wave] = (uint32_t)__popcll(qm);
    L.s_r[wave] = (uint32_t)__popcll(rm);
  }
  lds_barrier();
  uint32_t before = 0, total = 0, refl_total = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    before += k < wave ? L.s_q[k] : 0u;
    total += L.s_q[k];
    refl_total += L.s_r[k];
  }
  if (queue) {
    const uint32_t slot = before + (uint32_t)__popcll(qm & ((1ull << lane) - 1ull));
    L.id[slot] = (int32_t)w;
    L.dl[0][slot] = dl[0];
    L.dl[1][slot] = dl[1];
    L.dl[2][slot] = dl[2];
  }
  if (threadIdx.x == 0) {
    if (refl_total) counter_add(&V.counters[kWallReflect], (unsigned long long)refl_total);
    if (total) counter_add(&V.counters[kNearSurface], (unsigned long long)total);
  }
  lds_barrier();
  // the queued walkers, packed into the first waves of the block
  if (threadIdx.x < total) {
    const R q[3] = {L.dl[0][threadIdx.x], L.dl[1][threadIdx.x], L.dl[2][threadIdx.x]};
    walk_near_surface<P>(V, t, L.id[threadIdx.x], q);
  }
}

// A walker with a candidate particle at either end of its step: the full
// classification against the particles at t+1 (types I-IV), Algorithm 1 and
// Algorithm 2 for type IV, the refill of type II, then walls and
// renormalisation.  dl is the step drawn by the fast path.
template <int P>
__device__ void walk_near_surface(const DomView& V, uint64_t t, int64_t w, const typename Store<P>::O dl[3]) {
  using R = typename Store<P>::O;
  const int ps = pose_slot(t);
  const int nx = V.n[0], ny = V.n[1];
  const auto off = gp((const R*)V.woff);
  {
    const uint32_t lc = (uint32_t)gp(V.wcell)[w];
    const uint32_t q1 = fdiv(lc, V.dx);
    const int cz = (int)fdiv(q1, V.dy);
    int c[3] = {(int)(lc - q1 * (uint32_t)nx), (int)q1 - cz * ny, cz};
    const R o[3] = {off[w], off[V.nw + w], off[2 * V.nw + w]};
    R xf[3], xn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xf[a] = o[a] + dl[a];
      xn[a] = xf[a];
    }
    const int jb = inside_any<R>(V, ps, c, xf);
    if (jb >= 0) {
      const int ja = inside_any<R>(V, ps, c, o);
      if (ja < 0) {
        // type IV: no-flux boundary, Algorithm 1 then Algorithm 2
        counter_add(&V.counters[kType4], 1ull);
        R s;
        bool done = false;
        if (bisect<R>(V, ps, jb, c, o, dl, (R)0, (R)1, V.max_bisect, s)) {
          R xi[3], g[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) xi[a] = o[a] + s * dl[a];
          particle_grad_at<R>(V, ps, jb, c, xi, g);
          const R gn = sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]);
          if (gn > (R)0) {
            R nv[3], ti[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              nv[a] = g[a] / gn;
              ti[a] = xf[a] - xi[a];
            }
            const R dt = (ti[0] * nv[0] + ti[1] * nv[1]) + ti[2] * nv[2];
#pragma unroll
            for (int a = 0; a < 3; ++a) xn[a] = xi[a] + (ti[a] - ((R)2 * dt) * nv[a]);
            if (inside_any<R>(V, ps, c, xn) >= 0) {
              counter_add(&V.counters[kReturned], 1ull);
#pragma unroll
              for (int a = 0; a < 3; ++a) xn[a] = o[a];
            }
            done = true;
          }
        }
        if (!done) {
          counter_add(&V.counters[kBisectFail], 1ull);
#pragma unroll
          for (int a = 0; a < 3; ++a) xn[a] = o[a];
        }
      } else {
        // type II: refill (push out along -grad M, random point in the
        // sqrt(2D) half-ball on the outer side of the surface)
        counter_add(&V.counters[kType2], 1ull);
        R g[3];
        particle_grad_at<R>(V, ps, jb, c, xf, g);
        const R gn = sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]);
        bool fallback = true;
        if (gn > (R)0) {
          const R no[3] = {(-g[0]) / gn, (-g[1]) / gn, (-g[2]) / gn};
          R s = (R)0.5;
          const R lim = (R)(2.0 * gp(V.parts)[jb].rb);
          R xe[3];
          for (;;) {
#pragma unroll
            for (int a = 0; a < 3; ++a) xe[a] = xf[a] + s * no[a];
            if (!(particle_M_at<R>(V, ps, jb, c, xe) >= (R)1) || !(s < lim)) break;
            s = (R)2 * s;
          }
          if (particle_M_at<R>(V, ps, jb, c, xe) < (R)1) {
            R ss;
            if (bisect<R>(V, ps, jb, c, xf, no, s, (R)0, V.max_bisect, ss)) {
              R xs[3];
#pragma unroll
              for (int a = 0; a < 3; ++a) xs[a] = xf[a] + ss * no[a];
              const uint32_t id = (uint32_t)gp(V.wid)[w];
              const U4 r1 = philox4x32_10(id, (uint32_t)t, 1u, 0u, V.key0, V.key1);
              const U4 r2 = philox4x32_10(id, (uint32_t)t, 2u, 0u, V.key0, V.key1);
              R v[3];
              if constexpr (P == P64) {
                double v0, v1, v2;
                gauss3(r1, v0, v1, v2);
                v[0] = v0; v[1] = v1; v[2] = v2;
              } else {
                float v0, v1, v2;
                gauss3_fast(r1, v0, v1, v2);
                v[0] = v0; v[1] = v1; v[2] = v2;
              }
              const R vn = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
#pragma unroll
              for (int a = 0; a < 3; ++a) v[a] = v[a] / vn;
              if ((v[0] * no[0] + v[1] * no[1]) + v[2] * no[2] < (R)0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) v[a] = -v[a];
              }
              double mx = unit_open(r2.x);
              if (unit_open(r2.y) > mx) mx = unit_open(r2.y);
              if (unit_open(r2.z) > mx) mx = unit_open(r2.z);
              R rr;
              if constexpr (P == P64) rr = V.sD * mx;
              else rr = V.sD_f * (R)mx;
#pragma unroll
              for (int a = 0; a < 3; ++a) xn[a] = xs[a] + rr * v[a];
            } else {
              counter_add(&V.counters[kBisectFail], 1ull);
#pragma unroll
              for (int a = 0; a < 3; ++a) xn[a] = xe[a];
            }
            bool bad = inside_any<R>(V, ps, c, xn) >= 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              if (bad || !V.bc[a]) continue;
              const R lo = (R)(1.0 - (double)c[a]);
              const R hi = (R)((double)(V.n[a] - 1) - (double)c[a]);
              if (xn[a] < lo || xn[a] >= hi) bad = true;
            }
            if (bad) {
#pragma unroll
              for (int a = 0; a < 3; ++a) xn[a] = xe[a];
            }
            fallback = inside_any<R>(V, ps, c, xn) >= 0;
          }
        }
        if (fallback) {
          counter_add(&V.counters[kRefillFallback], 1ull);
#pragma unroll
          for (int a = 0; a < 3; ++a) xn[a] = xf[a];
        }
      }
    }
    if (!finite3<R>(xn)) {
      counter_add(&V.counters[kReturned], 1ull);
#pragma unroll
      for (int a = 0; a < 3; ++a) xn[a] = o[a];
    }
    if (reflect_walls<R>(V, c, xn)) {
      counter_add(&V.counters[kWallReflect], 1ull);
      if (outside_walls<R>(V, c, xn) || inside_any<R>(V, ps, c, xn) >= 0) {
        counter_add(&V.counters[kReturned], 1ull);
#pragma unroll
        for (int a = 0; a < 3; ++a) xn[a] = o[a];
      }
    }
    store_walker<R>(V, w, c, xn);
  }
}

}  // namespace rwmi
