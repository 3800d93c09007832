// Device-side building blocks shared by the kernels of librwmi.
//
// Every double-precision routine here follows one fixed sequence of IEEE
// operations (compiled with -ffp-contract=off for the FP64 path), so that the
// FP64 mode reproduces any other IEEE implementation of the same sequence bit
// for bit.  The low-precision modes reuse the routines templated on float.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace rwmi {

// ------------------------------------------------------------------ lattice
// D3Q19 (Sec. 2.3): rest, +-x, +-y, +-z, then the twelve edge diagonals in
// opposite pairs.  Opposite of i > 0 is i + 1 for odd i, i - 1 for even i.
constexpr int kQ = 19;
constexpr int kEx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kEy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kEz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__host__ __device__ constexpr int opp_dir(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// Component a of e_i for a direction known only at run time, from the table
// packed two bits per direction into a constant (0, 1 or 2 for -1): indexing
// the constexpr arrays at run time would make the kernel copy them to
// per-lane scratch memory.
constexpr uint64_t pack_dirs(const int (&e)[kQ]) {
  uint64_t b = 0;
  for (int i = 0; i < kQ; ++i) b |= (uint64_t)(e[i] < 0 ? 2 : e[i]) << (2 * i);
  return b;
}
constexpr uint64_t kExBits = pack_dirs(kEx), kEyBits = pack_dirs(kEy), kEzBits = pack_dirs(kEz);
__host__ __device__ __forceinline__ int dir_comp(uint64_t bits, int i) {
  const int v = (int)((bits >> (2 * i)) & 3ull);
  return v == 2 ? -1 : v;
}
__host__ __device__ __forceinline__ int ex_of(int i) { return dir_comp(kExBits, i); }
__host__ __device__ __forceinline__ int ey_of(int i) { return dir_comp(kEyBits, i); }
__host__ __device__ __forceinline__ int ez_of(int i) { return dir_comp(kEzBits, i); }
__host__ __device__ constexpr int comp(int i, int a) { return a == 0 ? kEx[i] : (a == 1 ? kEy[i] : kEz[i]); }
template <typename R>
__host__ __device__ constexpr R weight(int i) {
  return i == 0 ? R(1.0) / R(3.0) : (i <= 6 ? R(1.0) / R(18.0) : R(1.0) / R(36.0));
}

// Distribution layouts.  Two lattices (streamed from HBM) are stored in
// tiles: kTile consecutive nodes (x fastest) form a tile, which holds the
// kTile values of direction 0, then of direction 1, ... up to 18, so that a
// wave's 19 loads and 19 stores fall in a few contiguous regions of memory
// instead of 19 planes one lattice apart.  A lattice streamed in place (small
// enough to run from the memory-side cache) keeps one plane of N values per
// direction, whose cheaper neighbour addressing keeps the in-place kernel
// free of register spills.  Allocations hold ceil(N / kTile) whole tiles, at
// most 2^32 - 1 elements (a domain has at most kMaxNodes nodes), so element
// indices are 32-bit.
constexpr int kTileShift = 8;
constexpr uint32_t kTile = 1u << kTileShift;
constexpr int64_t kMaxNodes = ((int64_t)0xFFFFFFFF / (kQ * (int64_t)kTile)) * (int64_t)kTile;
// Element of direction `slot` of node n: slot * fstride + fnode(n).  Kernels
// form it as a wave-uniform base (slot * fstride) plus the per-node offset.
__host__ __device__ __forceinline__ uint32_t fnode(bool tiled, uint32_t n) {
  return tiled ? ((n >> kTileShift) * (uint32_t)kQ << kTileShift) + (n & (kTile - 1u)) : n;
}
__host__ __device__ __forceinline__ uint32_t fstride(bool tiled, uint32_t N) { return tiled ? kTile : N; }
__host__ __device__ __forceinline__ size_t fidx(bool tiled, int slot, uint32_t n, uint32_t N) {
  return (size_t)slot * fstride(tiled, N) + fnode(tiled, n);
}
__host__ __device__ __forceinline__ uint64_t f_elems(int64_t N) {
  return (uint64_t)((N + (int64_t)kTile - 1) >> kTileShift) * (uint64_t)kQ * (uint64_t)kTile;
}

constexpr int kMaxParticles = 64;
constexpr int kCounters = 8;
// kDemSkin: a coupled particle moved farther in one step than the margin of
// the contact candidate list (its contacts of that step may be missed).
enum CounterIdx { kType2 = 0, kType4, kBisectFail, kRefillFallback, kReturned, kWallReflect, kNearSurface, kDemSkin };
// Pose table record of one particle: centre, velocity, angular velocity.
constexpr int kPoseRec = 9;
// Interpolated bounce-back: the particle bits of a node's status byte.
constexpr uint8_t kSolidBits = 0x7F;
// 2^48: the fixed-point scale of the hydrodynamic force and torque sums on
// coupled particles (sums of at most 2^15 in magnitude).
constexpr double kForceFix = 281474976710656.0;
constexpr int kMaskBlock = 4;  // edge of a coarse block of the walker cull mask
// The start cell's coarse mask word also covers the end of any walker step
// with |dl| <= kMaskReach on every axis: the prologue dilates each coarse
// block by that much.
constexpr float kMaskReach = 1.0f;
// The fast path's float bounding-sphere filter enlarges every radius by this
// many lattice units, which covers the float rounding of its test.
constexpr float kSphereMargin = 0.05f;

// Precision tags
enum Prec { P64 = 0, P32 = 1, P16 = 2, PB16 = 3 };

// floor(n / d) for 0 <= n < 2^31 and 1 <= d < 2^31 by one 32x32->64 multiply
// and a shift (Granlund-Montgomery, round-up multiplier with N = 31 bits):
// l = ceil(log2 d), s = 31 + l, m = ceil(2^s / d) < 2^32.
struct FastDiv {
  uint32_t m;
  uint32_t s;
  int32_t d;
  int32_t pad;
};
inline FastDiv make_fastdiv(int32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < (unsigned long long)d) ++l;
  FastDiv f;
  f.s = 31 + l;
  f.m = (uint32_t)(((1ull << f.s) + (unsigned long long)d - 1ull) / (unsigned long long)d);
  f.d = d;
  f.pad = 0;
  return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((unsigned long long)n * (unsigned long long)f.m) >> f.s);
}

// Per-particle record in device memory.
struct DevParticle {
  double c0[3], amp[3], vel[3];
  double period, phase;
  double rb;      // bounding radius: M <= 1 beyond it
  double epscut2; // (rb + 3/4)^2: the solid fraction is 0 beyond rb + 3/4
  double shell2;  // (sqrt(K) + 3/4)^2, K the sum of the weights: the solid
                  // fraction is 0 farther than sqrt(K) + 3/4 from every
                  // control point
  double maskr;   // rb + 0.5, radius used to build the walker cull mask
  int32_t motion, nc, ctrl0, pad;
};

// Everything a kernel needs to know about one domain.  Lives in device memory
// (one per domain, or an array for a batch); constant across steps.
struct DomView {
  FastDiv dx, dy, dmx, dmy;  // division by nx, ny, mb[0], mb[1]
  int32_t n[3];
  int32_t bc[3];
  int32_t mb[3];     // coarse mask blocks per axis
  int32_t np;        // particles
  int64_t N;         // nodes
  int64_t nw;        // walkers
  int32_t prec;
  int32_t inplace;   // 1: one lattice streamed in place (slots by step parity); 0: two lattices
  int32_t has_force;
  int32_t max_bisect;
  uint32_t key0, key1;
  double tau, omega, tm, cfree;   // 1/tau, tau - 1/2, 1 - 1/(2 tau)
  double F[3], rho0, sD;          // force, initial density, sqrt(2D)
  float omega_f, tm_f, cfree_f, rho0_f, sD_f, F_f[3], halfF_f[3];
  float eF_f[kQ];                 // e_i . F per direction (float collision)
  double wu[3][2][3];             // wall velocity [axis][lo/hi][component]
  float wu_f[3][2][3];
  void* fA;                       // distributions (fidx): parity 0 source (two lattices) or the lattice (in place)
  void* fB;                       // distributions, parity 1 source (two lattices only)
  void* u[2];                     // (ux, uy, uz) per node (3 U), written by step t into [t & 1]
  void* rho;                      // density per node, written by the last fluid step of a group
  const DevParticle* parts;
  const double* ctrl;             // 4 per control point: bx, by, bz, k (body frame)
  const float* ctrl_f;            // the same in float (low-precision modes)
  const double* ctrlr[3];         // per pose slot s: control points at the pose P(s) of
  const float* ctrlr_f[3];        // the slot's fluid step (offsets rotated with the
                                  // particle; all three are ctrl when nothing rotates)
  double* pose[3];                // per step t, slot t mod 3: [2][np][kPoseRec] (c, v, w)
                                  // at t and t+1
  float* sph[3];                  // per step t, slot t mod 3: [np][4] walker filter spheres at
                                  // t+1: centre, (rb + 1/2 + kSphereMargin)^2
  uint64_t* tstep;                // [0] steps completed before the current launch group
  unsigned long long* mask[3];    // per step t, slot t mod 3: coarse cull mask at P(t+1)
  unsigned long long* fcull[3];   // per step t, slot t mod 3: bit p set when particle p's
                                  // solid-fraction support at P(t) meets fluid block b
  int32_t* wcell;                 // walker cell index
  void* woff;                     // walker offsets SoA [3][nw] (double or float)
  int32_t* wimg;                  // walker image counts SoA [3][nw]
  int32_t* wid;                   // walker id held by slot i (Philox counter, read-back order)
  int32_t* winv;                  // slot of walker id w (inverse of wid; built for read-outs)
  unsigned long long* counters;   // kCounters
  uint32_t* occ;                  // occupancy per node
  int32_t ibb;                    // interpolated bounce-back coupling instead of partially
                                  // saturated cells (two lattices only)
  uint8_t* smap[2];               // IBB: node status of the fluid update of step t in
                                  // [t & 1]: 0 fluid, p + 1 inside particle p
  uint32_t* solid_list[2];        // IBB: the nodes solid at the fluid update of step t,
                                  // in [t & 1], in no particular order
  uint32_t* solid_count;          // IBB: [2], their numbers
  unsigned long long dem_mask;    // bit p: particle p moves by Newton-Euler (two-way coupled)
  unsigned long long* dem_acc;    // [np][6] hydrodynamic force and torque of the running
                                  // fluid step, two's-complement sums in units of 2^-48
};

// Global-address-space view of a pointer loaded from memory, so that accesses
// compile to global_* (not flat_*) instructions.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gp(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Block barrier that orders LDS only: global memory operations in flight
// stay in flight across it (no wait for outstanding loads or stores).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Event counter increment: a relaxed device-scope atomic on the global
// address space (a global, not a flat, atomic instruction).
__device__ __forceinline__ void counter_add(unsigned long long* p, unsigned long long v) {
  __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long*)p, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// Constant-address-space view of a pointer to data that no block of the
// running launch writes: wave-uniform loads through it compile to scalar
// loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* kp(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// Step t of a launch: the domain's step counter at the start of the launch
// group plus the launch's offset k within the group.
__device__ __forceinline__ uint64_t step_of(const DomView& V, int32_t k) {
  return (uint64_t)((int64_t)kp(V.tstep)[0] + k);
}

// Slot of the pose table and cull mask of step t.  Three slots: one launch
// writes those of step t+1 while its fluid blocks read step t's and its
// walker blocks step t-1's.
__device__ __forceinline__ int pose_slot(uint64_t t) { return (int)(t % 3ull); }

// Work map of a multi-domain launch: block b of the grid belongs to domain d
// with boff[d] <= b < boff[d + 1].
__device__ __forceinline__ int find_domain(const int32_t* __restrict__ boff, int nd, int b) {
  int lo = 0, hi = nd;  // invariant boff[lo] <= b < boff[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (boff[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1) {
  // each 32x32 -> 64-bit product as one 64-bit multiply, which compiles to a
  // single v_mad_u64_u32 instead of separate low and high multiplies
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// Uniform in (0, 1): (r + 1/2) 2^-32, exact in double.
__device__ __forceinline__ double unit_open(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }

// ln(u) for normal u in (0, 1] using only +,-,*,/ on exactly split
// mantissa/exponent: m in (sqrt(1/2), sqrt(2)], s = (m-1)/(m+1),
// ln m = 2s + 2s s^2 (1/3 + s^2/5 + ... + s^20/21), then e ln 2 in two parts.
__device__ __forceinline__ double log_unit(double u) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(u);
  int e = (int)((bits >> 52) & 0x7ffull) - 1023;
  double m = __longlong_as_double((long long)((bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
  if (m > 0x1.6a09e667f3bcdp+0) {
    m = m * 0.5;
    e = e + 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  constexpr double c[10] = {1.0 / 21.0, 1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0,
                            1.0 / 11.0, 1.0 / 9.0,  1.0 / 7.0,  1.0 / 5.0,  1.0 / 3.0};
  double p = c[0];
#pragma unroll
  for (int j = 1; j < 10; ++j) p = p * z + c[j];
  const double t = 2.0 * s;
  const double lm = t + (t * z) * p;
  const double de = (double)e;
  return de * 0x1.62e42feep-1 + (de * 0x1.a39ef35793c76p-33 + lm);
}

// Taylor polynomials on [0, pi/4] (degree 17 for sine, 16 for cosine), Horner
// in x^2 with the signed reciprocal factorials.
__device__ __forceinline__ double sin_taylor(double x) {
  const double z = x * x;
  constexpr double c[8] = {1.0 / 355687428096000.0, -1.0 / 1307674368000.0, 1.0 / 6227020800.0,
                           -1.0 / 39916800.0,       1.0 / 362880.0,          -1.0 / 5040.0,
                           1.0 / 120.0,             -1.0 / 6.0};
  double p = c[0];
#pragma unroll
  for (int j = 1; j < 8; ++j) p = p * z + c[j];
  return x + (x * z) * p;
}
__device__ __forceinline__ double cos_taylor(double x) {
  const double z = x * x;
  constexpr double c[8] = {1.0 / 20922789888000.0, -1.0 / 87178291200.0, 1.0 / 479001600.0,
                           -1.0 / 3628800.0,       1.0 / 40320.0,        -1.0 / 720.0,
                           1.0 / 24.0,             -1.0 / 2.0};
  double p = c[0];
#pragma unroll
  for (int j = 1; j < 8; ++j) p = p * z + c[j];
  return 1.0 + z * p;
}

// sin and cos of 2 pi u, u in [0, 1): quarter-turn q = floor(4u) and the
// fraction f = 4u - q are exact; f > 1/2 is folded to 1 - f (exact) with sine
// and cosine swapped; the quarter turns are applied by sign/swap.
__device__ __forceinline__ void sincos_turns(double u, double& s, double& c) {
  const double t4 = 4.0 * u;
  const double qd = floor(t4);
  const double f = t4 - qd;
  const int q = ((int)qd) & 3;
  double a, b;  // sin, cos of the folded angle
  if (f <= 0.5) {
    const double x = f * 0x1.921fb54442d18p+0;
    a = sin_taylor(x);
    b = cos_taylor(x);
  } else {
    const double x = (1.0 - f) * 0x1.921fb54442d18p+0;
    a = cos_taylor(x);
    b = sin_taylor(x);
  }
  if (q == 0) { s = a; c = b; }
  else if (q == 1) { s = b; c = -a; }
  else if (q == 2) { s = -a; c = -b; }
  else { s = -b; c = a; }
}

// Three standard normals from one Philox block (Box-Muller on (r0, r1) and
// (r2, r3)).
__device__ __forceinline__ void gauss3(const U4& r, double& z0, double& z1, double& z2) {
  const double R0 = sqrt(-2.0 * log_unit(unit_open(r.x)));
  double s, c;
  sincos_turns(unit_open(r.y), s, c);
  z0 = R0 * c;
  z1 = R0 * s;
  const double R2 = sqrt(-2.0 * log_unit(unit_open(r.z)));
  sincos_turns(unit_open(r.w), s, c);
  z2 = R2 * c;
}

// Float normals for the low-precision modes: the same Philox words and the
// same Box-Muller map, with the hardware base-2 log, turn-scaled sine/cosine
// and square root (close to the double normals, not bit-identical).
__device__ __forceinline__ float unit_open_f(uint32_t r) { return (float)unit_open(r); }
__device__ __forceinline__ void gauss3_fast(const U4& r, float& z0, float& z1, float& z2) {
  constexpr float m2ln2 = -1.3862943611198906f;  // -2 ln 2
  const float R0 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(unit_open_f(r.x)));
  const float a = unit_open_f(r.y);
  z0 = R0 * __builtin_amdgcn_cosf(a);
  z1 = R0 * __builtin_amdgcn_sinf(a);
  const float R2 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(unit_open_f(r.z)));
  z2 = R2 * __builtin_amdgcn_cosf(unit_open_f(r.w));
}

// a / b: IEEE division in double, hardware reciprocal in float.
template <typename R> __device__ __forceinline__ R qdiv(R a, R b);
template <> __device__ __forceinline__ double qdiv<double>(double a, double b) { return a / b; }
template <> __device__ __forceinline__ float qdiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// sqrt: IEEE in double, hardware square root in float.
template <typename R> __device__ __forceinline__ R qsqrt(R a);
template <> __device__ __forceinline__ double qsqrt<double>(double a) { return sqrt(a); }
template <> __device__ __forceinline__ float qsqrt<float>(float a) { return __builtin_amdgcn_sqrtf(a); }

// ------------------------------------------------------------------ motion
// Pose (centre, velocity) of particle p at integer step t.
__device__ __forceinline__ void particle_pose(const DevParticle& p, uint64_t t, double c[3], double v[3]) {
  if (p.motion == 1) {
    double ph = (double)t / p.period + p.phase;
    ph = ph - floor(ph);
    double s, co;
    sincos_turns(ph, s, co);
    const double w = 0x1.921fb54442d18p+2 / p.period;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = p.c0[a] + p.amp[a] * s;
      v[a] = (p.amp[a] * w) * co;
    }
  } else if (p.motion == 2) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = p.c0[a] + p.vel[a] * (double)t;
      v[a] = p.vel[a];
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = p.c0[a];
      v[a] = 0.0;
    }
  }
}

// ------------------------------------------------------------------ geometry
// Displacement from a particle centre cp to (cell + x) along one axis, with
// the minimum image r - L floor(r / L + 1/2) on periodic axes.  In float the
// image is r - L rint(r / L) with a hardware reciprocal: it can differ from
// the FP64 choice only where |r| is within rounding of L / 2, where both
// images are equally far.
template <typename R>
__device__ __forceinline__ R axis_disp(int periodic, int L, int cell, double cp, R x) {
  R r = (R)((double)cell - cp) + x;
  if (periodic) {
    const R Lr = (R)L;
    r = r - Lr * rintf(r * __builtin_amdgcn_rcpf(Lr));
  }
  return r;
}
template <>
__device__ __forceinline__ double axis_disp<double>(int periodic, int L, int cell, double cp, double x) {
  double r = ((double)cell - cp) + x;
  if (periodic) {
    const double Lr = (double)L;
    r = r - Lr * floor(r / Lr + 0.5);
  }
  return r;
}

// Metaball value M = sum k_i / |d - b_i|^2 in control-point order (Eq. 3);
// +inf at a control point.
template <typename R, typename PT>
__device__ __forceinline__ R metaball_value(PT ctrl, int nc, R dx, R dy, R dz) {
  // A control point at distance 0 gives k / 0 = +inf (k > 0), so M = +inf
  // with no early exit; without a branch the loop unrolls and several control
  // points are loaded at once.
  R M = (R)0;
#pragma unroll 4
  for (int i = 0; i < nc; ++i) {
    const auto q = ctrl + 4 * i;
    const R rx = dx - (R)q[0], ry = dy - (R)q[1], rz = dz - (R)q[2];
    const R r2 = (rx * rx + ry * ry) + rz * rz;
    M = M + qdiv<R>((R)q[3], r2);
  }
  return M;
}

// Gradient of M (Eq. 17): sum -2 k_i (d - b_i) / |d - b_i|^4.
template <typename R, typename PT>
__device__ __forceinline__ void metaball_grad(PT ctrl, int nc, R dx, R dy, R dz, R g[3]) {
  g[0] = g[1] = g[2] = (R)0;
#pragma unroll 4
  for (int i = 0; i < nc; ++i) {
    const auto q = ctrl + 4 * i;
    const R rx = dx - (R)q[0], ry = dy - (R)q[1], rz = dz - (R)q[2];
    const R r2 = (rx * rx + ry * ry) + rz * rz;
    const R f = qdiv<R>((R)-2 * (R)q[3], r2 * r2);
    g[0] = g[0] + f * rx;
    g[1] = g[1] + f * ry;
    g[2] = g[2] + f * rz;
  }
}

// ------------------------------------------------------------------ storage
template <int P> struct Store;
template <> struct Store<P64> { using S = double; using C = double; using U = double; using O = double; };
template <> struct Store<P32> { using S = float; using C = float; using U = float; using O = float; };
template <> struct Store<P16> { using S = __half; using C = float; using U = float; using O = float; };
template <> struct Store<PB16> { using S = __hip_bfloat16; using C = float; using U = float; using O = float; };

__device__ __forceinline__ float to_c(__half h) { return __half2float(h); }
__device__ __forceinline__ float to_c(__hip_bfloat16 h) { return __bfloat162float(h); }
__device__ __forceinline__ float to_c(float h) { return h; }
__device__ __forceinline__ double to_c(double h) { return h; }
template <typename S> __device__ __forceinline__ S from_c(float v);
template <> __device__ __forceinline__ __half from_c<__half>(float v) { return __float2half_rn(v); }
template <> __device__ __forceinline__ __hip_bfloat16 from_c<__hip_bfloat16>(float v) { return __float2bfloat16(v); }
template <> __device__ __forceinline__ float from_c<float>(float v) { return v; }
template <typename S> __device__ __forceinline__ S from_d(double v) { return (S)v; }

// Raw storage words: 16-bit modes are moved as unsigned short and converted
// in registers (round to nearest even on the way out).
template <typename S> struct Raw { using T = S; };
template <> struct Raw<__half> { using T = unsigned short; };
template <> struct Raw<__hip_bfloat16> { using T = unsigned short; };
template <typename S> __device__ __forceinline__ typename Store<P32>::C raw_in(typename Raw<S>::T b);
template <> __device__ __forceinline__ float raw_in<float>(float b) { return b; }
template <> __device__ __forceinline__ float raw_in<__half>(unsigned short b) { return __half2float(__ushort_as_half(b)); }
template <> __device__ __forceinline__ float raw_in<__hip_bfloat16>(unsigned short b) {
  return __uint_as_float((uint32_t)b << 16);
}
template <typename S> __device__ __forceinline__ typename Raw<S>::T raw_out(float v);
template <> __device__ __forceinline__ float raw_out<float>(float v) { return v; }
template <> __device__ __forceinline__ unsigned short raw_out<__half>(float v) {
  return __half_as_ushort(__float2half_rn(v));
}
template <> __device__ __forceinline__ unsigned short raw_out<__hip_bfloat16>(float v) {
  // round to nearest even on the upper 16 bits (inputs are finite)
  const uint32_t u = __float_as_uint(v);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Control points at the pose of slot s, in the arithmetic precision of a mode.
template <typename R> __device__ __forceinline__ const R* ctrl_of(const DomView& V, int s);
template <> __device__ __forceinline__ const double* ctrl_of<double>(const DomView& V, int s) { return V.ctrlr[s]; }
template <> __device__ __forceinline__ const float* ctrl_of<float>(const DomView& V, int s) { return V.ctrlr_f[s]; }
// Slot of the pose P(t+1) that the walkers of step t (pose table slot ps) move against.
__device__ __forceinline__ int next_slot(int ps) { return ps == 2 ? 0 : ps + 1; }
// metaball sums read control points through a global pointer
template <typename T> using gconst = const __attribute__((address_space(1))) T*;

}  // namespace rwmi
