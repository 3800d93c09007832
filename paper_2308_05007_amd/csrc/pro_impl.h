// Walker-side prologue of a step: particle poses and the coarse walker cull
// mask (a block function of the fused step launch).
#pragma once
#include "dev_common.h"
#include "lbm_impl.h"

namespace rwmi {

// The cull words need only a superset of the particles that meet a block: a
// walker with a candidate bit runs the exact sphere test, a fluid node the
// exact support test.  So the prologue tests in float, with every radius
// enlarged by kCullMargin lattice units, which covers the float rounding of
// coordinates far beyond any lattice that fits in memory.
constexpr float kCullMargin = 0.05f;

// Lower bound on the distance from coordinate c to the interval [a, b] on an
// axis of length L (circular when periodic; invL = 1 / L).
__device__ __forceinline__ float gap_lb(int periodic, float L, float invL, float a, float b, float c) {
  if (!periodic) return fmaxf(fmaxf(a - c, c - b), 0.0f);
  float m = c - 0.5f * (a + b);
  m = m - L * rintf(m * invL);
  return fmaxf(fabsf(m) - 0.5f * (b - a), 0.0f);
}

// Does the sphere (centre c, squared enlarged radius r2) meet the box
// [lo, hi]?
__device__ __forceinline__ bool sphere_meets(const DomView& V, const float lo[3], const float hi[3], const float c[3],
                                             float r2) {
  float g2 = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float L = (float)V.n[a];
    const float g = gap_lb(!V.bc[a], L, 1.0f / L, lo[a], hi[a], c[a]);
    g2 += g * g;
  }
  return g2 <= r2;
}

// Bits p, among the candidates `cand`, of the particles (centres c[p],
// squared enlarged radii r2[p]) whose sphere meets the box [lo, hi].
__device__ __forceinline__ unsigned long long box_bits(const DomView& V, const float lo[3], const float hi[3],
                                                       const float (*c)[3], const float* r2, unsigned long long cand) {
  unsigned long long bits = 0ull;
  while (cand) {
    const int p = __ffsll((long long)cand) - 1;
    cand &= cand - 1ull;
    if (sphere_meets(V, lo, hi, c[p], r2[p])) bits |= 1ull << p;
  }
  return bits;
}

// Node-centre box of the fluid blocks [f0, f1] (bs nodes each).
__device__ __forceinline__ void fluid_blocks_box(const DomView& V, int bs, int64_t f0, int64_t f1, float lo[3],
                                                 float hi[3]) {
  const uint32_t N = (uint32_t)V.N;
  const uint32_t n0 = (uint32_t)f0 * (uint32_t)bs;
  const uint32_t e = (uint32_t)(f1 + 1) * (uint32_t)bs;
  const uint32_t n1 = (e < N ? e : N) - 1;
  int blo[3], bhi[3];
  node_range_box(V, n0, n1, blo, bhi);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = (float)blo[a] + 0.5f;
    hi[a] = (float)bhi[a] + 0.5f;
  }
}

// Box of the coarse mask blocks [m0, m1], dilated by the walker mask reach
// (the word also serves the end point of a step of at most kMaskReach per
// axis from any cell of the block) and extended to infinity beyond wall
// planes.
__device__ __forceinline__ void mask_blocks_box(const DomView& V, int64_t m0, int64_t m1, float lo[3], float hi[3]) {
  int blo[3], bhi[3];
  index_range_box((uint32_t)m0, (uint32_t)m1, V.dmx, V.dmy, V.mb[0], V.mb[1], blo, bhi);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int e = (bhi[a] + 1) * kMaskBlock;
    lo[a] = (float)(blo[a] * kMaskBlock) - kMaskReach;
    hi[a] = (float)(e < V.n[a] ? e : V.n[a]) + kMaskReach;
    if (V.bc[a]) {
      if (blo[a] == 0) lo[a] = -1e30f;
      if (bhi[a] == V.mb[a] - 1) hi[a] = 1e30f;
    }
  }
}

struct ProLds {
  float c1[kMaxParticles][3];  // centres at t + 1
  float rm2[kMaxParticles];    // squared walker mask radius, enlarged
  float c0[kMaxParticles][3];  // centres at t
  float rc2[kMaxParticles];    // squared solid-fraction support radius, enlarged
  unsigned long long cand_f, cand_m;  // particles that meet the block's whole range
};

// Prologue of step t (table slot t mod 3).  Block 0 of a domain writes the
// poses P(t), P(t+1) into pose[slot] and the walkers' filter spheres at t+1
// into sph[slot].  Thread i of the prologue blocks
// (i = lb blockDim + threadIdx.x) builds
// - word i of the coarse walker mask at P(t+1) in mask[slot]: bit p set when
//   the sphere (c_p(t+1), rb_p + 1/2) meets coarse block i dilated by
//   kMaskReach (and extended to infinity beyond wall planes), and possibly
//   for particles just beyond;
// - the cull word of fluid block i (blocks of bs nodes) at P(t) in
//   fcull[slot]: bit p set when the support (c_p(t), rb_p + 3/4) meets the
//   block's node centres, and possibly for particles just beyond.
// Each thread tests only the particles that meet the bounding box of its
// prologue block's whole range of words.  Every thread of the block calls
// it.
//
// With coupled particles (`dem`) the poses are not known ahead: the particle
// update after the fluid step of t - 1 has written P(t) into the pose table
// (slot t mod 3 for the fluid of t, slot t - 1 mod 3 for the walkers of
// t - 1) together with the filter spheres.  The prologue of t then builds
// only the masks at P(t): the fluid cull words of slot t mod 3 and the
// walker mask of slot t - 1 mod 3.
__device__ __forceinline__ void prologue_block(const DomView& V, int lb, uint64_t t, int bs, ProLds& L, bool dem) {
  const int ps = pose_slot(t);
  const int psm = dem ? (ps == 0 ? 2 : ps - 1) : ps;  // slot of the walker mask
  const int tid = threadIdx.x;
  if (tid < V.np) {
    const DevParticle& P = V.parts[tid];
    double c0[3], v0[3], c1[3], v1[3];
    if (dem) {
      const auto pt = gp((const double*)V.pose[ps]) + kPoseRec * tid;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        c0[a] = pt[a];
        c1[a] = pt[a];
      }
    } else {
      particle_pose(P, t, c0, v0);
      particle_pose(P, t + 1, c1, v1);
    }
    if (lb == 0 && !dem) {
      double* pt = V.pose[ps] + kPoseRec * tid;
      double* pn = V.pose[ps] + kPoseRec * (V.np + tid);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pt[a] = c0[a];
        pt[3 + a] = v0[a];
        pt[6 + a] = 0.0;
        pn[a] = c1[a];
        pn[3 + a] = v1[a];
        pn[6 + a] = 0.0;
      }
      // the walkers' filter sphere at t+1, one 16-byte record
      using F4 = float __attribute__((ext_vector_type(4)));
      const float rs = (float)P.maskr + kSphereMargin;
      const F4 sp = {(float)c1[0], (float)c1[1], (float)c1[2], rs * rs};
      *gp((F4*)V.sph[ps] + tid) = sp;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      L.c1[tid][a] = (float)c1[a];
      L.c0[tid][a] = (float)c0[a];
    }
    const float rm = (float)P.maskr + kCullMargin;
    // interpolated bounce-back: a node within rb + sqrt(2) can have a solid
    // neighbour, so the fluid cull reaches rb + 2
    const float rc = (V.ibb ? (float)P.rb + 2.0f : (float)sqrt(P.epscut2)) + kCullMargin;
    L.rm2[tid] = rm * rm;
    L.rc2[tid] = rc * rc;
  }
  if (V.np == 0) return;  // uniform: no barrier is skipped by part of the block
  // candidates of the whole block (a superset for each of its words): the
  // particles whose sphere meets the bounding box of the block's fluid blocks
  // or coarse blocks; wave 0 holds every particle (at most 64)
  const int64_t c0i = (int64_t)lb * blockDim.x;
  const int64_t c1i = c0i + blockDim.x - 1;
  const int64_t nfb = (V.N + bs - 1) / bs;
  const int64_t nmb = (int64_t)V.mb[0] * V.mb[1] * V.mb[2];
  if (tid < 64) {
    bool inf = false, inm = false;
    if (tid < V.np) {
      float lo[3], hi[3];
      if (c0i < nfb) {
        fluid_blocks_box(V, bs, c0i, c1i < nfb ? c1i : nfb - 1, lo, hi);
        const float c[3] = {L.c0[tid][0], L.c0[tid][1], L.c0[tid][2]};
        inf = sphere_meets(V, lo, hi, c, L.rc2[tid]);
      }
      if (V.nw > 0 && c0i < nmb) {
        mask_blocks_box(V, c0i, c1i < nmb ? c1i : nmb - 1, lo, hi);
        const float c[3] = {L.c1[tid][0], L.c1[tid][1], L.c1[tid][2]};
        inm = sphere_meets(V, lo, hi, c, L.rm2[tid]);
      }
    }
    const unsigned long long bf = __ballot(inf), bm = __ballot(inm);
    if (tid == 0) {
      L.cand_f = bf;
      L.cand_m = bm;
    }
  }
  lds_barrier();
  const int64_t cb = c0i + tid;
  if (cb < nfb) {
    float lo[3], hi[3];
    fluid_blocks_box(V, bs, cb, cb, lo, hi);
    V.fcull[ps][cb] = box_bits(V, lo, hi, L.c0, L.rc2, L.cand_f);
  }
  if (V.nw == 0 || cb >= nmb) return;
  float lo[3], hi[3];
  mask_blocks_box(V, cb, cb, lo, hi);
  V.mask[psm][cb] = box_bits(V, lo, hi, L.c1, L.rm2, L.cand_m);
}

}  // namespace rwmi
