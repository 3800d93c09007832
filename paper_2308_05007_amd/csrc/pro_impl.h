// Walker-side prologue of a step: particle poses and the coarse walker cull
// mask (a block function of the fused step launch).
#pragma once
#include "dev_common.h"
#include "lbm_impl.h"

namespace rwmi {

// Circular or plain gap between coordinate c and the interval [a, b].
__device__ __forceinline__ double gap_to(int periodic, int L, double a, double b, double c) {
  if (!periodic) {
    if (c < a) return a - c;
    if (c > b) return c - b;
    return 0.0;
  }
  const double hw = 0.5 * (b - a);
  if (2.0 * hw >= (double)L) return 0.0;
  double m = c - 0.5 * (a + b);
  m = m - (double)L * floor(m / (double)L + 0.5);
  const double g = fabs(m) - hw;
  return g > 0.0 ? g : 0.0;
}

struct ProLds {
  double c[kMaxParticles][3];   // centres at t + 1
  double r[kMaxParticles];      // walker mask radius
  double c0[kMaxParticles][3];  // centres at t
  double cut2[kMaxParticles];   // squared solid-fraction support radius
};

// Prologue of step t (table slot t mod 3).  Block 0 of a domain writes the
// poses P(t), P(t+1) into pose[slot].  Thread i of the prologue blocks
// (i = lb blockDim + threadIdx.x) builds
// - word i of the coarse walker mask at P(t+1) in mask[slot]: bit p set when
//   the sphere (c_p(t+1), rb_p + 1/2) meets coarse block i (extended to
//   infinity beyond wall planes);
// - the cull word of fluid block i (blocks of bs nodes) at P(t) in
//   fcull[slot].
// Every thread of the block calls it.
__device__ __forceinline__ void prologue_block(const DomView& V, int lb, uint64_t t, int bs, ProLds& L) {
  double (&sc)[kMaxParticles][3] = L.c;
  double (&sr)[kMaxParticles] = L.r;
  const int ps = pose_slot(t);
  const int tid = threadIdx.x;
  if (tid < V.np) {
    const DevParticle& P = V.parts[tid];
    double c0[3], v0[3], c1[3], v1[3];
    particle_pose(P, t, c0, v0);
    particle_pose(P, t + 1, c1, v1);
    if (lb == 0) {
      double* pt = V.pose[ps] + 6 * tid;
      double* pn = V.pose[ps] + 6 * (V.np + tid);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pt[a] = c0[a];
        pt[3 + a] = v0[a];
        pn[a] = c1[a];
        pn[3 + a] = v1[a];
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sc[tid][a] = c1[a];
      L.c0[tid][a] = c0[a];
    }
    sr[tid] = P.maskr;
    L.cut2[tid] = P.epscut2;
  }
  lds_barrier();
  if (V.np == 0) return;
  const int64_t cb = (int64_t)lb * blockDim.x + tid;
  const int64_t nfb = (V.N + bs - 1) / bs;
  if (cb < nfb) V.fcull[ps][cb] = fluid_cull_word(V, bs, cb, L.c0, L.cut2);
  const int64_t nmb = (int64_t)V.mb[0] * V.mb[1] * V.mb[2];
  if (V.nw == 0 || cb >= nmb) return;
  const int bidx[3] = {(int)(cb % V.mb[0]), (int)((cb / V.mb[0]) % V.mb[1]), (int)(cb / ((int64_t)V.mb[0] * V.mb[1]))};
  double lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = (double)(bidx[a] * kMaskBlock);
    const int e = (bidx[a] + 1) * kMaskBlock;
    hi[a] = (double)(e < V.n[a] ? e : V.n[a]);
    if (V.bc[a]) {
      if (bidx[a] == 0) lo[a] = -1e300;
      if (bidx[a] == V.mb[a] - 1) hi[a] = 1e300;
    }
  }
  unsigned long long bits = 0ull;
  for (int p = 0; p < V.np; ++p) {
    double g2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double g = gap_to(!V.bc[a], V.n[a], lo[a], hi[a], sc[p][a]);
      g2 += g * g;
    }
    const double r = sr[p];
    if (g2 <= r * r * (1.0 + 1e-9) + 1e-9) bits |= (1ull << p);
  }
  V.mask[ps][cb] = bits;
}

}  // namespace rwmi
