// D3Q19 partially-saturated-cell BGK collide + pull-stream, one thread per
// node, one block per run of consecutive nodes (x fastest); a block function
// run by the fluid blocks of the fused step launch.
//
// Stored state between steps is the post-collision distribution f*(t-1)
// (layouts: fidx), with the moving-wall term of Eq. 23 already added to every
// population that will bounce off a wall node.  A step gathers
// f_i(x, t) = f*_i(x - e_i, t-1) (or the bounced f*_opp(i)(x) when x - e_i is
// a wall node), computes rho, u (Eq. 14-15, Guo half-force velocity), the
// solid fraction eps and solid velocity u_s of the metaballs in the block's
// cull word (Eq. 3, Eq. 17), collides (BGK, Eq. 12-13, Noble-Torczynski
// weighting, Guo source) and writes f*(t), plus (u, rho).  Two lattices: the
// node's own slots of the other buffer.  One lattice streamed in place: the
// node's opposite slots on even steps, the neighbours' slots on odd steps.
#pragma once
#include <type_traits>

#include "dev_common.h"

namespace rwmi {

constexpr int kLdsCtrl = 160;  // control points staged in LDS per block

// The particles culled for a block, in the collision's arithmetic type C.
template <typename C>
struct BlockParticles {
  int cnt;
  int id[kMaxParticles];
  int ctrl_off[kMaxParticles];  // offset in ctrl, or -1 to read global memory
  int ctrl0[kMaxParticles];     // first control point in the global table
  int nc[kMaxParticles];
  double c[kMaxParticles][3];
  double v[kMaxParticles][3];
  double w[kMaxParticles][3];  // angular velocity (coupled particles)
  int cslot;                   // pose slot of the control points
  C cut2[kMaxParticles];    // squared support radius about the centre
  C shell2[kMaxParticles];  // squared radius about each control point
  alignas(16) C ctrl[4 * kLdsCtrl];
};

// Circular (periodic) or plain distance from coordinate c to the node-centre
// interval [lo + 1/2, hi + 1/2].
__device__ __forceinline__ double interval_gap(int periodic, int L, int lo, int hi, double c) {
  const double a = (double)lo + 0.5, b = (double)hi + 0.5;
  if (!periodic) {
    if (c < a) return a - c;
    if (c > b) return c - b;
    return 0.0;
  }
  const double hw = 0.5 * (b - a);
  if (2.0 * hw >= (double)L - 1.0) return 0.0;
  double m = c - 0.5 * (a + b);
  m = m - (double)L * floor(m / (double)L + 0.5);
  const double g = fabs(m) - hw;
  return g > 0.0 ? g : 0.0;
}

// Exclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_exclusive_sum(int x) {
  const int lane = (int)(threadIdx.x & 63u);
  int s = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(s, d, 64);
    if (lane >= d) s += y;
  }
  return s - x;
}

// Bounding box, in node indices, of the node range [n0, n1] (x fastest).
// Bounding box, in grid indices, of the linear index range [n0, n1] of an
// nx x ny x nz grid (x fastest; dx, dy divide by nx, ny).
__device__ __forceinline__ void index_range_box(uint32_t n0, uint32_t n1, const FastDiv& dx, const FastDiv& dy, int nx,
                                                int ny, int lo[3], int hi[3]) {
  const uint32_t a0 = fdiv(n0, dx), a1 = fdiv(n1, dx);
  const int z0 = (int)fdiv(a0, dy), z1 = (int)fdiv(a1, dy);
  const int x0 = (int)(n0 - a0 * (uint32_t)nx), x1 = (int)(n1 - a1 * (uint32_t)nx);
  const int y0 = (int)a0 - z0 * ny, y1 = (int)a1 - z1 * ny;
  lo[2] = z0; hi[2] = z1;
  if (z0 == z1 && y0 == y1) { lo[0] = x0; hi[0] = x1; lo[1] = y0; hi[1] = y0; }
  else if (z0 == z1) { lo[0] = 0; hi[0] = nx - 1; lo[1] = y0; hi[1] = y1; }
  else { lo[0] = 0; hi[0] = nx - 1; lo[1] = 0; hi[1] = ny - 1; }
}

// Bounding box, in node indices, of the node range [n0, n1].
__device__ __forceinline__ void node_range_box(const DomView& V, uint32_t n0, uint32_t n1, int lo[3], int hi[3]) {
  index_range_box(n0, n1, V.dx, V.dy, V.n[0], V.n[1], lo, hi);
}

// Does the solid-fraction support (squared radius cut2 about centre pc) meet
// the node centres of the box [lo, hi]?
__device__ __forceinline__ bool support_meets_box(const DomView& V, const int lo[3], const int hi[3], const double pc[3],
                                                  double cut2) {
  double g2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double g = interval_gap(!V.bc[a], V.n[a], lo[a], hi[a], pc[a]);
    g2 += g * g;
  }
  return g2 <= cut2 * (1.0 + 1e-9) + 1e-9;
}

// Cull the particles at pose P(t) for the node range [n0, n1] of a block and
// stage their poses and control points in LDS (the moment reduction's
// blocks).  Called by every thread of the block; wave 0 does the work,
// taking the poses from the pose table of step t (written by the prologue of
// an earlier launch) or, with from_table false, computing them.  Ends with
// one block barrier.
template <typename C>
__device__ __forceinline__ void cull_block(const DomView& V, uint32_t n0, uint32_t n1, uint64_t t,
                                           BlockParticles<C>& sp, bool from_table) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    int lo[3], hi[3];
    node_range_box(V, n0, n1, lo, hi);
    bool keep = false;
    double pc[3] = {0, 0, 0}, pv[3] = {0, 0, 0}, pw[3] = {0, 0, 0};
    const auto P = gp(V.parts) + tid;
    if (tid < V.np) {
      if (from_table) {
        const auto pt = gp((const double*)V.pose[pose_slot(t)]) + kPoseRec * tid;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          pc[a] = pt[a];
          pv[a] = pt[3 + a];
          pw[a] = pt[6 + a];
        }
      } else {
        particle_pose(V.parts[tid], t, pc, pv);
      }
      keep = support_meets_box(V, lo, hi, pc, P->epscut2);
    }
    const unsigned long long m = __ballot(keep);
    const int nc = keep ? P->nc : 0;
    const int pre = wave_exclusive_sum(nc);  // kept particles in index order
    if (keep) {
      const int r = __popcll(m & ((1ull << tid) - 1ull));
      const int c0 = P->ctrl0;
      sp.id[r] = tid;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sp.c[r][a] = pc[a];
        sp.v[r][a] = pv[a];
        sp.w[r][a] = pw[a];
      }
      sp.cut2[r] = (C)P->epscut2;
      sp.shell2[r] = (C)P->shell2;
      sp.nc[r] = nc;
      sp.ctrl0[r] = c0;
      const bool fits = pre + nc <= kLdsCtrl;
      sp.ctrl_off[r] = fits ? pre : -1;
      if (fits) {
        const auto src = gp(ctrl_of<C>(V, pose_slot(t))) + 4 * c0;
        for (int i = 0; i < 4 * nc; ++i) sp.ctrl[4 * pre + i] = src[i];
      }
    }
    if (tid == 0) {
      sp.cnt = __popcll(m);
      sp.cslot = pose_slot(t);
    }
  }
  lds_barrier();
}

// Solid fraction of one particle at node nd: 1/2 + the signed distance
// estimate 2 M (sqrt M - 1) / |grad M|, clamped to [0, 1] (Eq. 3, Eq. 17).
//
// Nodes where the estimate is provably <= -3/4 get 0 without evaluating M.
// With all weights positive and r the distance to the nearest control point,
// M <= K / r^2 and |grad M| <= 2 M / r (K the sum of the weights).  If
// r >= sqrt(K) + 3/4 then 1 - sqrt(M) >= (3/4) / r (3/4 being 1/2 + 1/4), so
// the estimate is at most -(1 + 2/4) / 2 = -3/4 and the fraction is 0,
// however it is rounded.  The centre test uses the same bound with the
// bounding radius: beyond rb + 3/4 from the centre every control point is
// farther than sqrt(K) + 3/4.
template <typename R, typename PT>
__device__ __forceinline__ R eps_from_ctrl(PT ctrl, int nc, R dx, R dy, R dz, R shell2) {
  R rmin2 = (R)INFINITY;
#pragma unroll 4
  for (int i = 0; i < nc; ++i) {
    const auto q = ctrl + 4 * i;
    const R rx = dx - (R)q[0], ry = dy - (R)q[1], rz = dz - (R)q[2];
    const R r2 = (rx * rx + ry * ry) + rz * rz;
    rmin2 = r2 < rmin2 ? r2 : rmin2;
  }
  if (!(rmin2 < shell2)) return (R)0;
  // M (Eq. 3) and its gradient (Eq. 17) in one pass, each sum in control-point
  // order; the FP64 terms are the IEEE quotients k / r^2 and -2 k / r^4
  R M = (R)0, g0 = (R)0, g1 = (R)0, g2 = (R)0;
#pragma unroll 4
  for (int i = 0; i < nc; ++i) {
    const auto q = ctrl + 4 * i;
    const R rx = dx - (R)q[0], ry = dy - (R)q[1], rz = dz - (R)q[2];
    const R r2 = (rx * rx + ry * ry) + rz * rz;
    const R k = (R)q[3];
    R f;
    if constexpr (std::is_same<R, double>::value) {
      M = M + k / r2;
      f = ((R)-2 * k) / (r2 * r2);
    } else {
      const R inv = __builtin_amdgcn_rcpf(r2);
      const R tk = k * inv;
      M = M + tk;
      f = ((R)-2 * tk) * inv;
    }
    g0 = g0 + f * rx;
    g1 = g1 + f * ry;
    g2 = g2 + f * rz;
  }
  if (M == (R)INFINITY) return (R)1;  // on a control point
  const R gn = qsqrt<R>((g0 * g0 + g1 * g1) + g2 * g2);
  R e;
  if (gn == (R)0) {
    e = M >= (R)1 ? (R)1 : (R)0;
  } else {
    const R dist = qdiv<R>(((R)2 * M) * (qsqrt<R>(M) - (R)1), gn);
    e = dist == dist ? (R)0.5 + dist : (M >= (R)1 ? (R)1 : (R)0);
  }
  if (e < (R)0) e = (R)0;
  if (e > (R)1) e = (R)1;
  return e;
}

template <typename R>
__device__ __forceinline__ R node_eps(const DomView& V, const BlockParticles<R>& sp, int k, const int nd[3],
                                      R* dl = nullptr) {
  const R dx = axis_disp<R>(!V.bc[0], V.n[0], nd[0], sp.c[k][0], (R)0.5);
  const R dy = axis_disp<R>(!V.bc[1], V.n[1], nd[1], sp.c[k][1], (R)0.5);
  const R dz = axis_disp<R>(!V.bc[2], V.n[2], nd[2], sp.c[k][2], (R)0.5);
  if (dl) {
    dl[0] = dx;
    dl[1] = dy;
    dl[2] = dz;
  }
  const R r2c = (dx * dx + dy * dy) + dz * dz;
  if (!(r2c < sp.cut2[k])) return (R)0;
  const int off = sp.ctrl_off[k];
  if (off >= 0) return eps_from_ctrl<R>(sp.ctrl + 4 * off, sp.nc[k], dx, dy, dz, sp.shell2[k]);
  return eps_from_ctrl<R>(gp(ctrl_of<R>(V, sp.cslot)) + 4 * sp.ctrl0[k], sp.nc[k], dx, dy, dz, sp.shell2[k]);
}

// Velocity of a rigid body's surface at displacement dl from its centre:
// v + w x dl (coupled particles; the node's solid velocity, Sec. 2.4.3).
template <typename R>
__device__ __forceinline__ void rigid_velocity(const R w[3], const R dl[3], R v[3]) {
  v[0] = v[0] + (w[1] * dl[2] - w[2] * dl[1]);
  v[1] = v[1] + (w[2] * dl[0] - w[0] * dl[2]);
  v[2] = v[2] + (w[0] * dl[1] - w[1] * dl[0]);
}

// Solid fraction of particle p at node nd in a fluid block of step t, and the
// particle's velocity: pose from the pose table of slot ps, particle record
// and control points, all through wave-uniform scalar loads.
template <typename R>
__device__ __forceinline__ R node_eps_direct(const DomView& V, int ps, int p, const int nd[3], R v[3]) {
  const auto pt = kp((const double*)V.pose[ps]) + kPoseRec * p;
  const auto P = kp(V.parts) + p;
  v[0] = (R)pt[3];
  v[1] = (R)pt[4];
  v[2] = (R)pt[5];
  const R dx = axis_disp<R>(!V.bc[0], V.n[0], nd[0], pt[0], (R)0.5);
  const R dy = axis_disp<R>(!V.bc[1], V.n[1], nd[1], pt[1], (R)0.5);
  const R dz = axis_disp<R>(!V.bc[2], V.n[2], nd[2], pt[2], (R)0.5);
  const R r2c = (dx * dx + dy * dy) + dz * dz;
  if (!(r2c < (R)P->epscut2)) return (R)0;
  return eps_from_ctrl<R>(kp(ctrl_of<R>(V, ps)) + 4 * P->ctrl0, P->nc, dx, dy, dz, (R)P->shell2);
}

// The same for a coupled particle: the solid velocity at the node includes
// the rotation, v + w x dl, where the particle covers the node; dl is the
// node centre's displacement from the particle's centre.
template <typename R>
__device__ __forceinline__ R node_eps_coupled(const DomView& V, int ps, int p, const int nd[3], R v[3], R dl[3]) {
  const auto pt = kp((const double*)V.pose[ps]) + kPoseRec * p;
  const auto P = kp(V.parts) + p;
  v[0] = (R)pt[3];
  v[1] = (R)pt[4];
  v[2] = (R)pt[5];
  dl[0] = axis_disp<R>(!V.bc[0], V.n[0], nd[0], pt[0], (R)0.5);
  dl[1] = axis_disp<R>(!V.bc[1], V.n[1], nd[1], pt[1], (R)0.5);
  dl[2] = axis_disp<R>(!V.bc[2], V.n[2], nd[2], pt[2], (R)0.5);
  const R r2c = (dl[0] * dl[0] + dl[1] * dl[1]) + dl[2] * dl[2];
  if (!(r2c < (R)P->epscut2)) return (R)0;
  const R e = eps_from_ctrl<R>(kp(ctrl_of<R>(V, ps)) + 4 * P->ctrl0, P->nc, dl[0], dl[1], dl[2], (R)P->shell2);
  if (e > (R)0) {
    const R w[3] = {(R)pt[6], (R)pt[7], (R)pt[8]};
    rigid_velocity<R>(w, dl, v);
  }
  return e;
}

// e_i . v with zero components contributing nothing (left to right over x, y, z).
template <typename R>
__device__ __forceinline__ R edot(int i, R vx, R vy, R vz) {
  R s = (R)0;
  const int ex = ex_of(i), ey = ey_of(i), ez = ez_of(i);
  if (ex == 1) s = s + vx; else if (ex == -1) s = s - vx;
  if (ey == 1) s = s + vy; else if (ey == -1) s = s - vy;
  if (ez == 1) s = s + vz; else if (ez == -1) s = s - vz;
  return s;
}

// Wall node test for a neighbour at coordinate offsets (dx,dy,dz) of a fluid
// node at (x,y,z): returns the wall velocity slot (axis*2 + side) of the first
// wall axis on which the neighbour lies at index 0 or n-1, or -1.
__device__ __forceinline__ int wall_slot(const DomView& V, const int nd[3], int dx, int dy, int dz) {
  const int dd[3] = {dx, dy, dz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!V.bc[a] || dd[a] == 0) continue;
    const int c = nd[a] + dd[a];
    if (c == 0) return 2 * a;
    if (c == V.n[a] - 1) return 2 * a + 1;
  }
  return -1;
}

// Compile-time sum of the components of (ax, ay, az) picked by direction i
// (e_i . a with zero components skipped, left to right).
template <int i, typename R>
__device__ __forceinline__ R edot_c(R ax, R ay, R az) {
  R s = (R)0;
  if constexpr (kEx[i] == 1) s = s + ax; else if constexpr (kEx[i] == -1) s = s - ax;
  if constexpr (kEy[i] == 1) s = s + ay; else if constexpr (kEy[i] == -1) s = s - ay;
  if constexpr (kEz[i] == 1) s = s + az; else if constexpr (kEz[i] == -1) s = s - az;
  return s;
}

template <int I, int N_, typename F>
__device__ __forceinline__ void unroll(F&& f) {
  if constexpr (I < N_) {
    f(std::integral_constant<int, I>{});
    unroll<I + 1, N_>(f);
  }
}

// Lattice layouts of a step: two lattices, or one lattice streamed in place
// at an even or an odd step (the slots a step reads and writes).
enum Layout { kTwoLattices = 0, kInPlaceEven = 1, kInPlaceOdd = 2 };

// Linear offsets to the six face neighbours of a fluid node (periodic wrap)
// and whether the neighbour at -1 / +1 along an axis is a wall node.
struct Nbr {
  int dxm, dxp, dym, dyp, dzm, dzp;
  bool wxl, wxh, wyl, wyh, wzl, wzh;
};
__device__ __forceinline__ Nbr node_nbr(const DomView& V, int x, int y, int z) {
  const int nx = V.n[0], ny = V.n[1], nz = V.n[2];
  const int sxy = nx * ny;
  Nbr b;
  b.dxm = x > 0 ? -1 : nx - 1;
  b.dxp = x < nx - 1 ? 1 : -(nx - 1);
  b.dym = y > 0 ? -nx : (ny - 1) * nx;
  b.dyp = y < ny - 1 ? nx : -(ny - 1) * nx;
  b.dzm = z > 0 ? -sxy : (nz - 1) * sxy;
  b.dzp = z < nz - 1 ? sxy : -(nz - 1) * sxy;
  b.wxl = V.bc[0] && x == 1;
  b.wxh = V.bc[0] && x == nx - 2;
  b.wyl = V.bc[1] && y == 1;
  b.wyh = V.bc[1] && y == ny - 2;
  b.wzl = V.bc[2] && z == 1;
  b.wzh = V.bc[2] && z == nz - 2;
  return b;
}

// Offset to the neighbour x - e_i and whether it is a wall node.
template <int i>
__device__ __forceinline__ void upstream_of(const Nbr& b, bool& wall, int& delta) {
  constexpr int ex = kEx[i], ey = kEy[i], ez = kEz[i];
  wall = false;
  delta = 0;
  if constexpr (ex == 1) { wall |= b.wxl; delta += b.dxm; } else if constexpr (ex == -1) { wall |= b.wxh; delta += b.dxp; }
  if constexpr (ey == 1) { wall |= b.wyl; delta += b.dym; } else if constexpr (ey == -1) { wall |= b.wyh; delta += b.dyp; }
  if constexpr (ez == 1) { wall |= b.wzl; delta += b.dzm; } else if constexpr (ez == -1) { wall |= b.wzh; delta += b.dzp; }
}

// Nodes [lb BS, (lb + 1) BS) of a domain through step t in layout L (the
// domain's layout at t's parity); nt selects non-temporal stores, dens the
// store of the node densities as well.  Every thread of the block calls it.
// Exchange of population i with the solid, bo = B Om_i, and its share of
// the force on the solid: -e_i bo, summed per component in direction order.
template <int i, typename R>
__device__ __forceinline__ void solid_force(R bo, R& fx, R& fy, R& fz) {
  if constexpr (kEx[i] == 1) fx = fx - bo; else if constexpr (kEx[i] == -1) fx = fx + bo;
  if constexpr (kEy[i] == 1) fy = fy - bo; else if constexpr (kEy[i] == -1) fy = fy + bo;
  if constexpr (kEz[i] == 1) fz = fz - bo; else if constexpr (kEz[i] == -1) fz = fz + bo;
}

// ---------------------------------------------- interpolated bounce-back
// The paper's own coupling (Sec. 2.4.3, Eq. 23-27) in place of the partially
// saturated cells.  A node is solid while its centre is inside a particle
// (M_p >= 1, lowest index), else fluid; the status of step t's update is
// kept in smap[t & 1].  Step t gathers, for a fluid node x_f whose upstream
// node x_f - e_i was solid at the previous update (the populations it would
// pull were never produced), the bounced population of Eq. 23-25 at the
// geometry of that update; a node solid now stores its particle's rigid
// velocity and skips the collision; a node uncovered since the previous
// update starts from f^eq(rho0, u_new) (Eq. 27).

// v + w x dl from a pose record.
template <typename R, typename PT>
__device__ __forceinline__ void rigid_at(PT pt, const R dl[3], R up[3]) {
  up[0] = (R)pt[3];
  up[1] = (R)pt[4];
  up[2] = (R)pt[5];
  const R w[3] = {(R)pt[6], (R)pt[7], (R)pt[8]};
  rigid_velocity<R>(w, dl, up);
}

// Lowest particle among `bits` (index order) whose M >= 1 at the centre of
// node nd at the pose of slot ps, or -1; dl receives the node's offset from
// that particle's centre.
template <typename R>
__device__ __forceinline__ int solid_node(const DomView& V, int ps, unsigned long long bits, const int nd[3],
                                          R dl[3]) {
  while (bits) {
    const int p = __ffsll((long long)bits) - 1;
    bits &= bits - 1ull;
    const auto pt = kp((const double*)V.pose[ps]) + kPoseRec * p;
    const auto P = kp(V.parts) + p;
#pragma unroll
    for (int a = 0; a < 3; ++a) dl[a] = axis_disp<R>(!V.bc[a], V.n[a], nd[a], pt[a], (R)0.5);
    const R r2 = (dl[0] * dl[0] + dl[1] * dl[1]) + dl[2] * dl[2];
    const R rb = (R)P->rb;
    if (!(r2 < rb * rb)) continue;
    if (metaball_value<R>(kp(ctrl_of<R>(V, ps)) + 4 * P->ctrl0, P->nc, dl[0], dl[1], dl[2]) >= (R)1) return p;
  }
  return -1;
}

// f^eq of direction i (Eq. 13), in the stored form of precision P: the full
// value (FP64) or its deviation from w_i rho0.
template <int P>
__device__ __forceinline__ typename Store<P>::C feq_stored(const DomView& V, int i, typename Store<P>::C rho,
                                                           const typename Store<P>::C u[3]) {
  using R = typename Store<P>::C;
  const R eu = edot<R>(i, u[0], u[1], u[2]);
  const R u15 = (R)1.5 * ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  const R w = i == 0 ? weight<R>(0) : (i <= 6 ? weight<R>(1) : weight<R>(7));
  if constexpr (P == P64) return (w * rho) * ((((R)1 + (R)3 * eu) + (R)4.5 * (eu * eu)) - u15);
  else return w * ((rho - V.rho0_f) + rho * (eu * ((R)3 + (R)4.5 * eu) - u15));
}

// Eq. 23-25 for the link of fluid node id (coordinates nd) along e_i whose
// upstream node lies in particle p at the previous update (step t - 1):
// q from a bracketed regula falsi for the surface M_p = 1 on the segment from
// x_f towards the solid node; u_w the rigid velocity there; u_f, rho_f and
// the fluid-side neighbour's u_ff (u_f where that node is a wall or solid)
// from the update of t - 1; fso x_f's own post-collision population of the
// opposite direction.  DEM: the link's momentum exchange in its
// Galilean-invariant form, (e_o - u_w) fso - (e_i - u_w) f_i, and its torque
// about the particle's centre go to the block's accumulator.
// lctrl, when `lds`: every particle's control points at the pose of t - 1
// in LDS, at the offsets they have in the domain's table.
template <int P, bool DEM>
__device__ __forceinline__ typename Store<P>::C ibb_link(const DomView& V, uint64_t t, uint32_t id,
                                                                    int nx, int ny, int nz, int i, int p,
                                                                    typename Store<P>::C fso,
                                                                    unsigned long long* dacc,
                                                                    const typename Store<P>::C* lctrl = nullptr,
                                                                    bool lds = false) {
  using R = typename Store<P>::C;
  using U = typename Store<P>::U;
  const int nd[3] = {nx, ny, nz};
  const int o = opp_dir(i);
  const int eo[3] = {ex_of(o), ey_of(o), ez_of(o)};
  const int ps = pose_slot(t - 1);
  const auto pt = gp((const double*)V.pose[ps]) + kPoseRec * p;
  const auto Pp = gp(V.parts) + p;
  const int nc = Pp->nc;
  R d0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) d0[a] = axis_disp<R>(!V.bc[a], V.n[a], nd[a], pt[a], (R)0.5);
  // q: the root of 1 - M^(-1/2) in [0, 1] by the Illinois variant of regula
  // falsi (the bracket keeps a sign change), 10 steps in FP64, 6 in float
  constexpr int kSteps = P == P64 ? 10 : 6;
  const int p0 = __builtin_amdgcn_readfirstlane(p);
  const bool uni = __all(p == p0);
  // one particle for the whole wave: its control points through the scalar
  // cache (every step of the solve reads them)
  const auto ctrl_s = kp(ctrl_of<R>(V, ps)) + 4 * kp(V.parts)[p0].ctrl0;
  const int nc_s = kp(V.parts)[p0].nc;
  const int c0 = Pp->ctrl0;
  const auto ctrl_v = gp(ctrl_of<R>(V, ps)) + 4 * c0;
  auto phi = [&](R s) -> R {
    const R x[3] = {d0[0] + s * (R)eo[0], d0[1] + s * (R)eo[1], d0[2] + s * (R)eo[2]};
    R M;
    if (lds) M = metaball_value<R>(lctrl + 4 * c0, nc, x[0], x[1], x[2]);
    else M = uni ? metaball_value<R>(ctrl_s, nc_s, x[0], x[1], x[2]) : metaball_value<R>(ctrl_v, nc, x[0], x[1], x[2]);
    return (R)1 - qdiv<R>((R)1, qsqrt<R>(M));
  };
  R a0 = (R)0, b0 = (R)1;
  R fa = phi(a0), fb = phi(b0);
  for (int it = 0; it < kSteps; ++it) {
    if (fb == fa) break;
    const R c = b0 - fb * qdiv<R>(b0 - a0, fb - fa);
    const R fc = phi(c);
    if (fc == (R)0) {
      b0 = c;
      break;
    }
    if ((fc < (R)0) == (fb < (R)0)) fa = (R)0.5 * fa;
    else {
      a0 = b0;
      fa = fb;
    }
    b0 = c;
    fb = fc;
  }
  const R q = b0;
  const R dlw[3] = {d0[0] + q * (R)eo[0], d0[1] + q * (R)eo[1], d0[2] + q * (R)eo[2]};
  R uw[3];
  rigid_at<R>(pt, dlw, uw);
  const auto up = gp((const U*)V.u[(t - 1) & 1ull]);
  const R uf[3] = {(R)up[3ull * id], (R)up[3ull * id + 1], (R)up[3ull * id + 2]};
  const R rf = (R)gp((const U*)V.rho)[id];
  // x_ff = x_f + e_i
  int ff[3] = {nd[0] + ex_of(i), nd[1] + ey_of(i), nd[2] + ez_of(i)};
  bool fwall = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int n = V.n[a];
    if (V.bc[a]) {
      if (ff[a] <= 0 || ff[a] >= n - 1) fwall = true;
    } else {
      ff[a] = ff[a] < 0 ? ff[a] + n : (ff[a] >= n ? ff[a] - n : ff[a]);
    }
  }
  R uff[3] = {uf[0], uf[1], uf[2]};
  if (!fwall) {
    const uint32_t fid = (uint32_t)ff[0] + (uint32_t)V.n[0] * ((uint32_t)ff[1] + (uint32_t)V.n[1] * (uint32_t)ff[2]);
    if (!(gp(V.smap[(t - 1) & 1ull])[fid] & kSolidBits)) {
#pragma unroll
      for (int a = 0; a < 3; ++a) uff[a] = (R)up[3ull * fid + a];
    }
  }
  R ud[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R u1 = q <= (R)0.5 ? ((R)2 * q) * uf[a] + ((R)1 - (R)2 * q) * uff[a]
                             : (((R)1 - q) / q) * uf[a] + (((R)2 * q - (R)1) / q) * uw[a];
    const R u2 = (((R)1 - q) / ((R)1 + q)) * uff[a] + (((R)2 * q) / ((R)1 + q)) * uw[a];
    ud[a] = u1 / (R)3 + ((R)2 * u2) / (R)3;
  }
  const R w = o <= 6 ? weight<R>(1) : weight<R>(7);
  const R gneq = fso - feq_stored<P>(V, o, rf, uf);
  const R fi = (feq_stored<P>(V, o, rf, ud) + gneq) + (((R)6 * w) * rf) * edot<R>(i, uw[0], uw[1], uw[2]);
  if constexpr (DEM) {
    if ((V.dem_mask >> p) & 1ull) {
      // full populations for the exchange
      R fs = fso, fn = fi;
      if constexpr (P != P64) {
        fs = fs + w * V.rho0_f;
        fn = fn + w * V.rho0_f;
      }
      const R ei[3] = {(R)ex_of(i), (R)ey_of(i), (R)ez_of(i)};
      R F[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) F[a] = ((R)eo[a] - uw[a]) * fs - (ei[a] - uw[a]) * fn;
      const R T[3] = {dlw[1] * F[2] - dlw[2] * F[1], dlw[2] * F[0] - dlw[0] * F[2], dlw[0] * F[1] - dlw[1] * F[0]};
      unsigned long long* acc = dacc + 6 * p;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        atomicAdd(acc + k, (unsigned long long)__double2ll_rn((double)F[k] * kForceFix));
        atomicAdd(acc + 3 + k, (unsigned long long)__double2ll_rn((double)T[k] * kForceFix));
      }
    }
  }
  return fi;
}

// The link pass of step t, run before the step's fluid update.  For each
// node x_s that was solid at the previous update and each direction i whose
// downstream node x_f = x_s + e_i was fluid then (x_f's link along e_i), the
// bounced population of Eq. 23-25 (ibb_link) is written into slot i of x_s
// in the lattice step t pulls from, where x_f's gather finds it like any
// other population.  A solid node's own populations are not defined and
// each of its slots feeds one downstream node only, so no write meets a
// value that is still to be read; the inputs (x_f's own populations,
// velocities and densities of t - 1) belong to fluid nodes and are never
// written here.
//
// The work items are the (node, direction) pairs of the solid nodes the
// fluid update of t - 1 listed, 18 per node, spread over the launch's
// threads: every link runs in its own lane, and all of a step's links are
// in flight at once.  The control points of all particles are copied to LDS
// first when they fit (every step of a link's root search reads them).  The
// pass also clears the count of the list the fluid update of t fills.  DEM:
// the links' momentum exchange in the block's LDS accumulator, then in the
// step's.
constexpr unsigned kLinkGrid = 2048;  // blocks of the link pass
constexpr int kLinkCtrl = 1024;       // control points held in LDS

template <int P, bool DEM>
__global__ void __launch_bounds__(256) k_ibb_links(const DomView* __restrict__ views, int dom, int32_t j) {
  using S = typename Store<P>::S;
  using R = typename Store<P>::C;
  using SR = typename Raw<S>::T;
  __shared__ unsigned long long dacc[DEM ? 6 * kMaxParticles : 1];
  __shared__ R cl[4 * kLinkCtrl];
  const DomView& V = views[dom];
  if (V.np == 0) return;
  const uint64_t t = step_of(V, j);
  // the fluid update of t lists into [t & 1]; the pass of t - 1 has read it
  if (blockIdx.x == 0 && threadIdx.x == 0) V.solid_count[t & 1ull] = 0u;
  const uint32_t nn = V.solid_count[(t - 1) & 1ull];
  const uint64_t items = (uint64_t)nn * (kQ - 1);
  const uint64_t first = (uint64_t)blockIdx.x * 256u;
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  if (first >= items) return;  // uniform over the block
  const auto list = gp((const uint32_t*)V.solid_list[(t - 1) & 1ull]);
  const auto smp = gp((const uint8_t*)V.smap[(t - 1) & 1ull]);
  const auto src = gp((SR*)((t & 1ull) ? V.fB : V.fA));
  constexpr uint32_t FS = kTile;
  const auto plast = kp(V.parts) + (V.np - 1);
  const int nctl = plast->ctrl0 + plast->nc;
  const bool lds = nctl <= kLinkCtrl;
  if (lds) {
    const auto cg = gp(ctrl_of<R>(V, pose_slot(t - 1)));
    for (int k = threadIdx.x; k < 4 * nctl; k += 256) cl[k] = cg[k];
  }
  if constexpr (DEM)
    for (int k = threadIdx.x; k < 6 * kMaxParticles; k += 256) dacc[k] = 0ull;
  lds_barrier();
  for (uint64_t w = first + threadIdx.x; w < items; w += stride) {
    const uint32_t us = list[w / (kQ - 1)];
    const int i = 1 + (int)(w % (kQ - 1));
    const uint32_t q1 = fdiv(us, V.dx);
    const int zz = (int)fdiv(q1, V.dy);
    // downstream node x_f = x_s + e_i: a wall node is never updated
    int nd[3] = {(int)(us - q1 * (uint32_t)V.n[0]) + ex_of(i), (int)q1 - zz * V.n[1] + ey_of(i), zz + ez_of(i)};
    bool wall = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int m = V.n[a];
      if (V.bc[a]) wall = wall || nd[a] <= 0 || nd[a] >= m - 1;
      else nd[a] = nd[a] < 0 ? nd[a] + m : (nd[a] >= m ? nd[a] - m : nd[a]);
    }
    if (wall) continue;
    const uint32_t nid = (uint32_t)nd[0] + (uint32_t)V.n[0] * ((uint32_t)nd[1] + (uint32_t)V.n[1] * (uint32_t)nd[2]);
    if (smp[nid] & kSolidBits) continue;  // solid too: no link
    const uint8_t sb = smp[us] & kSolidBits;
    const SR raw = src[(size_t)opp_dir(i) * FS + fnode(true, nid)];
    R fso;
    if constexpr (P == P64) fso = raw;
    else fso = raw_in<S>(raw);
    const R v = ibb_link<P, DEM>(V, t, nid, nd[0], nd[1], nd[2], i, (int)sb - 1, fso, dacc, cl, lds);
    SR o;
    if constexpr (P == P64) o = v;
    else o = raw_out<S>(v);
    src[(size_t)i * FS + fnode(true, us)] = o;
  }
  if constexpr (DEM) {
    lds_barrier();
    for (int k = threadIdx.x; k < 6 * kMaxParticles; k += 256) {
      const unsigned long long v = dacc[k];
      if (((V.dem_mask >> (k / 6)) & 1ull) && v != 0ull) atomicAdd(V.dem_acc + k, v);
    }
  }
}

// One node of a fluid block.  DEM: two-way coupled particles; the momentum
// the solid term takes from the fluid at the node, -sum_i e_i B Om_i, is
// shared among the coupled particles that cover it in proportion to their
// solid fractions, and each share and its torque about the particle's centre
// go into the block's accumulator dacc ([64][6], LDS) in fixed point, so
// that the sums do not depend on the order of the nodes.
template <int P, int BS, int L, bool DEM, bool IBB>
__device__ __forceinline__ void fluid_node(const DomView& V, uint32_t lb, uint64_t t, bool nt, bool dens,
                                           unsigned long long* dacc) {
  using S = typename Store<P>::S;
  using R = typename Store<P>::C;
  constexpr bool exact = (P == P64);
  using SR = typename Raw<S>::T;
  // two lattices: read the parity-t buffer, write the other; in place (one
  // lattice): every access goes to fA, the slots depending on t's parity
  constexpr bool inplace = L != kTwoLattices;
  constexpr bool odd_ip = L == kInPlaceOdd;
  const bool odd = (t & 1ull) != 0;
  const auto src = gp((const SR*)((inplace || !odd) ? V.fA : V.fB));
  SR* dst0 = (SR*)((inplace || odd) ? V.fA : V.fB);
  // In place, dst equals src; hide that from the optimiser, which would
  // otherwise keep all 19 load addresses live until the stores instead of
  // recomputing them (this only moves a register value, no memory access).
  if constexpr (inplace) asm volatile("" : "+s"(dst0));
  const auto dst = gp(dst0);
  const uint32_t N = (uint32_t)V.N;
  const uint32_t FS = fstride(!inplace, N);  // elements between directions (layouts: fidx)
  const uint32_t n0 = lb * BS;
  const uint32_t id = n0 + threadIdx.x;
  const uint32_t idc = id < N ? id : n0;  // a valid node for the threads past the end
  const int nx = V.n[0], ny = V.n[1], nz = V.n[2];
  const int bx = V.bc[0], by = V.bc[1], bz = V.bc[2];
  const uint32_t q1 = fdiv(idc, V.dx);
  const int x = (int)(idc - q1 * (uint32_t)nx);
  const int z = (int)fdiv(q1, V.dy);
  const int y = (int)q1 - z * ny;
  // wall nodes are never updated
  const bool live = id < N && !((bx && (x == 0 || x == nx - 1)) || (by && (y == 0 || y == ny - 1)) ||
                                (bz && (z == 0 || z == nz - 1)));
  const int nd[3] = {x, y, z};
  const Nbr nb = node_nbr(V, x, y, z);
  const bool wxl = nb.wxl, wxh = nb.wxh, wyl = nb.wyl, wyh = nb.wyh, wzl = nb.wzl, wzh = nb.wzh;
  const bool near_wall = wxl | wxh | wyl | wyh | wzl | wzh;


  // ---- gather of f_i(x, t).  Two lattices: f*_i(x - e_i) of the last step
  // from slot i there, or the bounced f*_opp(i)(x) from the node's own slot
  // opp(i) when x - e_i is a wall node.  In place, even t: the node's own
  // slot i (the previous step pushed it there); odd t: f*_i(x - e_i) sits in
  // slot opp(i) of x - e_i (the previous step swapped it), or in the node's own
  // slot i when x - e_i is a wall node.
  R f[kQ];
  if (live) unroll<0, kQ>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    bool wall;
    int delta;
    upstream_of<i>(nb, wall, delta);
    int slot;
    uint32_t at;
    if constexpr (!inplace) {
      slot = wall ? opp_dir(i) : i;
      at = wall ? id : (uint32_t)((int)id + delta);
    } else if constexpr (!odd_ip) {
      slot = i;
      at = id;
    } else {
      slot = wall ? i : opp_dir(i);
      at = wall ? id : (uint32_t)((int)id + delta);
    }
    const SR raw = src[(size_t)slot * FS + fnode(!inplace, at)];
    if constexpr (exact) f[i] = raw;
    else f[i] = raw_in<S>(raw);
  });

  if (!live) return;
  if constexpr (IBB) {
    static_assert(!inplace, "interpolated bounce-back streams between two lattices");
    // a link whose upstream node was solid at the previous update was
    // gathered above like any other population: the link pass of this step
    // (k_ibb_links) wrote its bounced value into that node's slot.  A node
    // solid then has no populations of its own: it is solid now or refilled
    // below.
    const unsigned long long bprev = V.np > 0 ? kp(V.fcull[pose_slot(t - 1)])[lb] : 0ull;
    const uint8_t prev = bprev ? (uint8_t)(gp((const uint8_t*)V.smap[(t - 1) & 1ull])[id] & kSolidBits) : (uint8_t)0;
    // the node's own status at P(t)
    const int ps = pose_slot(t);
    const unsigned long long bits = V.np > 0 ? kp(V.fcull[ps])[lb] : 0ull;
    R dl[3];
    const int sn = bits ? solid_node<R>(V, ps, bits, nd, dl) : -1;
    gp(V.smap[t & 1ull])[id] = sn >= 0 ? (uint8_t)(sn + 1) : (uint8_t)0;
    {
      // a solid node joins the list the link pass of step t + 1 works
      // through (one atomic per wave)
      const bool app = sn >= 0;
      const unsigned long long bal = __ballot(app);
      if (bal) {
        const int lane = (int)__lane_id();
        const int leader = __ffsll((long long)bal) - 1;
        uint32_t base = 0u;
        if (lane == leader) base = atomicAdd(V.solid_count + (t & 1ull), (uint32_t)__popcll(bal));
        base = (uint32_t)__shfl((int)base, leader);
        if (app) gp(V.solid_list[t & 1ull])[base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = id;
      }
    }
    if (sn >= 0) {
      R up[3];
      rigid_at<R>(kp((const double*)V.pose[ps]) + kPoseRec * sn, dl, up);
      using U = typename Store<P>::U;
      const auto u = gp((U*)V.u[t & 1ull]) + 3ull * (uint64_t)id;
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = (U)up[a];
      gp((U*)V.rho)[id] = (U)V.rho0;
      return;
    }
    if (prev) {  // uncovered since the previous update: Eq. 27
      const int pp = (int)prev - 1;
      const auto pt = kp((const double*)V.pose[ps]) + kPoseRec * pp;
      R d[3], un[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) d[a] = axis_disp<R>(!V.bc[a], V.n[a], nd[a], pt[a], (R)0.5);
      rigid_at<R>(pt, d, un);
      R r0;
      if constexpr (exact) r0 = V.rho0;
      else r0 = V.rho0_f;
#pragma unroll
      for (int i = 0; i < kQ; ++i) f[i] = feq_stored<P>(V, i, r0, un);
    }
  }
  // ---- solid fraction and solid velocity of the node, over the particles
  // whose support meets the block (cull word from the prologue), in index
  // order
  R es = (R)0, unx = (R)0, uny = (R)0, unz = (R)0;
  unsigned long long cbits = 0ull;  // DEM: coupled particles that cover the node
  if (!IBB && V.np > 0) {
    const int ps = pose_slot(t);
    unsigned long long bits = kp(V.fcull[ps])[lb];
    while (bits) {
      const int p = __ffsll((long long)bits) - 1;
      bits &= bits - 1ull;
      R v[3];
      R e;
      if constexpr (DEM) {
        if ((V.dem_mask >> p) & 1ull) {
          R dl[3];
          e = node_eps_coupled<R>(V, ps, p, nd, v, dl);
          if (e > (R)0) cbits |= 1ull << p;
        } else {
          e = node_eps_direct<R>(V, ps, p, nd, v);
        }
      } else {
        e = node_eps_direct<R>(V, ps, p, nd, v);
      }
      es = es + e;
      unx = unx + e * v[0];
      uny = uny + e * v[1];
      unz = unz + e * v[2];
    }
  }
  const R eps = es < (R)1 ? es : (R)1;
  const bool solid = eps > (R)0;

  // ---- moments (Eq. 14-15; Guo half-force velocity)
  R rho, drho;
  if constexpr (exact) {
    rho = (R)0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) rho = rho + f[i];
    drho = rho;
  } else {
    drho = (R)0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) drho = drho + f[i];
    rho = V.rho0_f + drho;
  }
  R jx = (R)0, jy = (R)0, jz = (R)0;
  unroll<0, kQ>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (kEx[i] == 1) jx = jx + f[i]; else if constexpr (kEx[i] == -1) jx = jx - f[i];
    if constexpr (kEy[i] == 1) jy = jy + f[i]; else if constexpr (kEy[i] == -1) jy = jy - f[i];
    if constexpr (kEz[i] == 1) jz = jz + f[i]; else if constexpr (kEz[i] == -1) jz = jz - f[i];
  });
  R ux, uy, uz;
  if constexpr (exact) {
    ux = (jx + 0.5 * V.F[0]) / rho;
    uy = (jy + 0.5 * V.F[1]) / rho;
    uz = (jz + 0.5 * V.F[2]) / rho;
  } else {
    const R ir = (R)1 / rho;
    ux = (jx + V.halfF_f[0]) * ir;
    uy = (jy + V.halfF_f[1]) * ir;
    uz = (jz + V.halfF_f[2]) * ir;
  }

  // ---- BGK relaxation (Eq. 12-13), Noble-Torczynski weighting where eps > 0
  R omega, tm, cfree;
  if constexpr (exact) { omega = V.omega; tm = V.tm; cfree = V.cfree; }
  else { omega = V.omega_f; tm = V.tm_f; cfree = V.cfree_f; }
  const R uu15 = (R)1.5 * ((ux * ux + uy * uy) + uz * uz);
  R B = (R)0, A = omega, Cf = cfree;
  if (solid) {
    B = (eps * tm) / (((R)1 - eps) + tm);
    A = ((R)1 - B) * omega;
    Cf = ((R)1 - B) * ((R)1 - (R)0.5 * omega);
  }
  R usx = (R)0, usy = (R)0, usz = (R)0, us15 = (R)0;
  if (solid) {
    usx = unx / es;
    usy = uny / es;
    usz = unz / es;
    us15 = (R)1.5 * ((usx * usx + usy * usy) + usz * usz);
  }
  R Fx, Fy, Fz;
  if constexpr (exact) { Fx = V.F[0]; Fy = V.F[1]; Fz = V.F[2]; }
  else { Fx = V.F_f[0]; Fy = V.F_f[1]; Fz = V.F_f[2]; }
  const R uF = (ux * Fx + uy * Fy) + uz * Fz;
  const bool force = V.has_force != 0;

  // equilibria: exact form (w rho)(((1 + 3 eu) + 4.5 eu^2) - 1.5 uu); the
  // shifted form feq - w rho0 = w (drho + rho (3 eu + 4.5 eu^2 - 1.5 uu))
  auto feq = [&](auto ic, R eu, R u15) -> R {
    constexpr int i = decltype(ic)::value;
    if constexpr (exact) return (weight<R>(i) * rho) * ((((R)1 + (R)3 * eu) + (R)4.5 * (eu * eu)) - u15);
    else return weight<R>(i) * (drho + rho * (eu * ((R)3 + (R)4.5 * eu) - u15));
  };
  // Guo source S_i = w_i [3 (e_i - u).F + 9 (e_i.u)(e_i.F)]
  auto guo = [&](auto ic, R eu) -> R {
    constexpr int i = decltype(ic)::value;
    const R eF = edot_c<i, R>(Fx, Fy, Fz);
    if constexpr (exact) {
      R emF = (R)0;
      emF = emF + ((R)kEx[i] - ux) * Fx;
      emF = emF + ((R)kEy[i] - uy) * Fy;
      emF = emF + ((R)kEz[i] - uz) * Fz;
      return weight<R>(i) * ((R)3 * emF + ((R)9 * eu) * eF);
    } else {
      return weight<R>(i) * ((R)3 * (eF - uF) + (R)9 * eu * eF);
    }
  };
  // moving-wall term for a population headed for a wall node (Eq. 23 form),
  // added now so that the next gather only has to bounce it
  auto wall_term = [&](auto jc, R& v) {
    constexpr int j = decltype(jc)::value;
    constexpr int i = opp_dir(j);
    constexpr int ex = kEx[j], ey = kEy[j], ez = kEz[j];
    int ws = -1;  // wall slot of the first wall axis the neighbour x + e_j lies on
    if constexpr (ex == -1) { if (wxl) ws = 0; } else if constexpr (ex == 1) { if (wxh) ws = 1; }
    if constexpr (ey == -1) { if (ws < 0 && wyl) ws = 2; } else if constexpr (ey == 1) { if (ws < 0 && wyh) ws = 3; }
    if constexpr (ez == -1) { if (ws < 0 && wzl) ws = 4; } else if constexpr (ez == 1) { if (ws < 0 && wzh) ws = 5; }
    if (ws >= 0) {
      const int a = ws >> 1, side = ws & 1;
      R wx, wy, wz;
      if constexpr (exact) { wx = V.wu[a][side][0]; wy = V.wu[a][side][1]; wz = V.wu[a][side][2]; }
      else { wx = V.wu_f[a][side][0]; wy = V.wu_f[a][side][1]; wz = V.wu_f[a][side][2]; }
      v = v + (((R)6 * weight<R>(i)) * rho) * edot_c<i, R>(wx, wy, wz);
    }
  };
  // ---- store of f*_j(x, t).  Two lattices: slot j of the node.  In place,
  // even t: slot opp(j) of the node (swap); odd t: slot j of x + e_j (push),
  // or slot opp(j) of the node itself when x + e_j is a wall node (bounce).
  // x + e_j is the upstream neighbour of direction opp(j).  The push targets
  // are recomputed from an opaque copy of the node's coordinates, so that the
  // optimiser does not keep the gather's 19 addresses (the same locations)
  // live through the collision.
  Nbr nbs = nb;
  uint32_t ids = id;
  if constexpr (odd_ip) {
    int cx = x, cy = y, cz = z;
    asm volatile("" : "+v"(cx), "+v"(cy), "+v"(cz), "+v"(ids));
    nbs = node_nbr(V, cx, cy, cz);
  }
  auto put = [&](auto jc, R v) {
    constexpr int j = decltype(jc)::value;
    SR w;
    if constexpr (exact) w = v;
    else w = raw_out<S>(v);
    int slot = j;
    uint32_t at = id;
    if constexpr (inplace) {
      if constexpr (!odd_ip) {
        slot = opp_dir(j);
      } else {
        bool wall;
        int delta;
        upstream_of<opp_dir(j)>(nbs, wall, delta);
        slot = wall ? opp_dir(j) : j;
        at = wall ? ids : (uint32_t)((int)ids + delta);
      }
    }
    if (nt) __builtin_nontemporal_store(w, &dst[(size_t)slot * FS + fnode(!inplace, at)]);
    else dst[(size_t)slot * FS + fnode(!inplace, at)] = w;
  };

  // Float collision, folded: with e_o = -e_i and w_o = w_i the relaxed,
  // forced population of an opposite pair is
  //   (1 - A) f_i + w_i (S +- D),
  //   S = K0 + eu (K2 eu + K3 eF),  D = eu K1 + K4 eF,
  // eu = e_i.u, eF = e_i.F, K0 = A (drho - rho 1.5 u.u) - 3 Cf u.F,
  // K1 = 3 A rho, K2 = 4.5 A rho, K3 = 9 Cf, K4 = 3 Cf: the same BGK and Guo
  // terms as the FP64 form, in fewer operations.
  R omA = (R)0, K0 = (R)0, K1 = (R)0, K2 = (R)0, K3 = (R)0, K4 = (R)0;
  if constexpr (!exact) {
    omA = (R)1 - A;
    K1 = ((R)3 * A) * rho;
    K2 = ((R)4.5 * A) * rho;
    K0 = A * (drho - rho * uu15);
    if (force) {
      K3 = (R)9 * Cf;
      K4 = (R)3 * Cf;
      K0 = K0 - K4 * uF;
    }
  }
  // rest population
  {
    constexpr std::integral_constant<int, 0> i0{};
    R o0;
    if constexpr (exact) {
      const R fe0 = feq(i0, (R)0, uu15);
      o0 = f[0] - A * (f[0] - fe0);
      if (solid) o0 = o0 + B * ((f[0] - fe0) - (f[0] - feq(i0, (R)0, us15)));
      if (force) o0 = o0 + Cf * guo(i0, (R)0);
    } else {
      o0 = omA * f[0] + weight<R>(0) * K0;
      if (solid) o0 = o0 + B * (feq(i0, (R)0, us15) - feq(i0, (R)0, uu15));
    }
    put(i0, o0);
  }
  // opposite pairs (i, i+1): each pair is relaxed, exchanged with the solid,
  // forced and stored before the next, so few registers stay live
  R hfx = (R)0, hfy = (R)0, hfz = (R)0;  // DEM: force on the solid at the node
  unroll<0, 9>([&](auto pc) {
    constexpr int i = 1 + 2 * decltype(pc)::value;
    constexpr int o = i + 1;
    constexpr std::integral_constant<int, i> ic{};
    constexpr std::integral_constant<int, o> oc{};
    R vi, vo;
    if constexpr (exact) {
      const R eui = edot_c<i, R>(ux, uy, uz);
      const R euo = edot_c<o, R>(ux, uy, uz);
      const R fei = feq(ic, eui, uu15);
      const R feo = feq(oc, euo, uu15);
      vi = f[i] - A * (f[i] - fei);
      vo = f[o] - A * (f[o] - feo);
      if (solid) {
        const R fesi = feq(ic, edot_c<i, R>(usx, usy, usz), us15);
        const R feso = feq(oc, edot_c<o, R>(usx, usy, usz), us15);
        if constexpr (DEM) {
          const R boi = B * ((f[o] - feo) - (f[i] - fesi));
          const R boo = B * ((f[i] - fei) - (f[o] - feso));
          vi = vi + boi;
          vo = vo + boo;
          solid_force<i, R>(boi, hfx, hfy, hfz);
          solid_force<o, R>(boo, hfx, hfy, hfz);
        } else {
          vi = vi + B * ((f[o] - feo) - (f[i] - fesi));
          vo = vo + B * ((f[i] - fei) - (f[o] - feso));
        }
      }
      if (force) {
        vi = vi + Cf * guo(ic, eui);
        vo = vo + Cf * guo(oc, euo);
      }
    } else {
      // w S and w D with the weight folded into the node's constants (the
      // products are shared by the pairs of one weight class)
      const R eu = edot_c<i, R>(ux, uy, uz);
      constexpr R w = weight<R>(i);
      R S, D;
      if (force) {
        const R eF = kp(V.eF_f)[i];
        S = (w * K0) + eu * ((w * K2) * eu + (w * K3) * eF);
        D = eu * (w * K1) + (w * K4) * eF;
      } else {
        S = (w * K0) + eu * ((w * K2) * eu);
        D = eu * (w * K1);
      }
      vi = omA * f[i] + (S + D);
      vo = omA * f[o] + (S - D);
      if (solid) {
        // Noble-Torczynski exchange with the solid: B ((f_o - fe_o) - (f_i - fes_i))
        const R fei = feq(ic, eu, uu15);
        const R feo = feq(oc, -eu, uu15);
        const R eus = edot_c<i, R>(usx, usy, usz);
        const R fesi = feq(ic, eus, us15);
        const R feso = feq(oc, -eus, us15);
        if constexpr (DEM) {
          const R boi = B * ((f[o] - feo) - (f[i] - fesi));
          const R boo = B * ((f[i] - fei) - (f[o] - feso));
          vi = vi + boi;
          vo = vo + boo;
          solid_force<i, R>(boi, hfx, hfy, hfz);
          solid_force<o, R>(boo, hfx, hfy, hfz);
        } else {
          vi = vi + B * ((f[o] - feo) - (f[i] - fesi));
          vo = vo + B * ((f[i] - fei) - (f[o] - feso));
        }
      }
    }
    if (near_wall) {
      wall_term(ic, vi);
      wall_term(oc, vo);
    }
    put(ic, vi);
    put(oc, vo);
  });
  {
    // (ux, uy, uz): three consecutive U, merged into one store by the
    // compiler; the density only where a read-out may follow
    using U = typename Store<P>::U;
    const auto u = gp((U*)V.u[t & 1ull]) + 3ull * (uint64_t)id;
    const U v[3] = {(U)ux, (U)uy, (U)uz};
    if (nt) {
#pragma unroll
      for (int a = 0; a < 3; ++a) __builtin_nontemporal_store(v[a], u + a);
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = v[a];
    }
    if (dens) gp((U*)V.rho)[id] = (U)rho;
  }
  if constexpr (DEM) {
    // shares of the force and their torques, for each coupled particle
    // covering the node (its solid fraction and displacement recomputed:
    // the same arithmetic gives the same values)
    const int ps = pose_slot(t);
    unsigned long long bits = cbits;
    while (bits) {
      const int p = __ffsll((long long)bits) - 1;
      bits &= bits - 1ull;
      R v[3], dl[3];
      const R e = node_eps_coupled<R>(V, ps, p, nd, v, dl);
      const R share = e / es;
      const R F[3] = {share * hfx, share * hfy, share * hfz};
      const R T[3] = {dl[1] * F[2] - dl[2] * F[1], dl[2] * F[0] - dl[0] * F[2], dl[0] * F[1] - dl[1] * F[0]};
      unsigned long long* a = dacc + 6 * p;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        atomicAdd(a + k, (unsigned long long)__double2ll_rn((double)F[k] * kForceFix));
        atomicAdd(a + 3 + k, (unsigned long long)__double2ll_rn((double)T[k] * kForceFix));
      }
    }
  }
}

// Fluid block.  DEM: the coupled particles' force sums of the block in LDS,
// then in the step's accumulator.  The bounce-back coupling exchanges
// momentum at its links only, in the link pass: its fluid blocks take the
// non-DEM form.
template <int P, int BS, int L, bool DEM, bool IBB = false>
__device__ __forceinline__ void fluid_block(const DomView& V, uint32_t lb, uint64_t t, bool nt, bool dens,
                                            unsigned long long* dacc) {
  static_assert(!(DEM && IBB), "bounce-back links carry the momentum exchange");
  if constexpr (!DEM) {
    fluid_node<P, BS, L, false, IBB>(V, lb, t, nt, dens, dacc);
  } else {
    for (int k = threadIdx.x; k < 6 * kMaxParticles; k += BS) dacc[k] = 0ull;
    lds_barrier();
    fluid_node<P, BS, L, true, IBB>(V, lb, t, nt, dens, dacc);
    lds_barrier();
    // the block's sums into the step's accumulator (two's-complement adds:
    // exact, in any order)
    unsigned long long bits = V.np > 0 ? kp(V.fcull[pose_slot(t)])[lb] : 0ull;
    bits &= V.dem_mask;
    for (int k = threadIdx.x; k < 6 * kMaxParticles; k += BS) {
      const unsigned long long v = dacc[k];
      if (((bits >> (k / 6)) & 1ull) && v != 0ull) atomicAdd(V.dem_acc + k, v);
    }
  }
}

// Initial stored state: the gather of step 0 reads f = feq(rho0, u0) at
// every fluid node (with two lattices, populations that bounce are set to the
// value they must arrive with); u = u0 in both velocity buffers (wall nodes
// carry the wall velocity) and rho = rho0.
template <int P>
__global__ void k_init(const DomView* __restrict__ views, int dom, double u0x, double u0y, double u0z) {
  using S = typename Store<P>::S;
  using U = typename Store<P>::U;
  const DomView& V = views[dom];
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= V.N) return;
  const int nx = V.n[0], ny = V.n[1];
  const int nd[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((int64_t)nx * ny))};
  int wslot = -1;
  for (int a = 0; a < 3 && wslot < 0; ++a)
    if (V.bc[a] && (nd[a] == 0 || nd[a] == V.n[a] - 1)) wslot = 2 * a + (nd[a] == 0 ? 0 : 1);
  const double rho0 = V.rho0;
  const double uu15 = 1.5 * ((u0x * u0x + u0y * u0y) + u0z * u0z);
  S* fA = (S*)V.fA;
  S* fB = (S*)V.fB;
  for (int j = 0; j < kQ; ++j) {
    // two lattices: slot j holds what streams into slot j's direction, so a
    // population that will bounce holds f^eq of the opposite direction; in
    // place (even layout) slot j of the node is f_j(x, 0) itself
    int i = j;
    if (!V.inplace && wslot < 0 && wall_slot(V, nd, kEx[j], kEy[j], kEz[j]) >= 0) i = opp_dir(j);
    const double eu = edot<double>(i, u0x, u0y, u0z);
    double fe = (weight<double>(i) * rho0) * (((1.0 + 3.0 * eu) + 4.5 * (eu * eu)) - uu15);
    if (P != P64) fe = fe - weight<double>(i) * rho0;
    const bool tiled = !V.inplace;
    fA[fidx(tiled, j, (uint32_t)id, (uint32_t)V.N)] = from_d<S>(fe);
    if (tiled) fB[fidx(tiled, j, (uint32_t)id, (uint32_t)V.N)] = from_d<S>(fe);
  }
  for (int b = 0; b < 2; ++b) {  // wall nodes keep these values in both buffers
    U* u = (U*)V.u[b] + 3 * id;
    if (wslot >= 0) {
      const int a = wslot >> 1, side = wslot & 1;
      u[0] = (U)V.wu[a][side][0];
      u[1] = (U)V.wu[a][side][1];
      u[2] = (U)V.wu[a][side][2];
    } else {
      u[0] = (U)u0x;
      u[1] = (U)u0y;
      u[2] = (U)u0z;
    }
  }
  ((U*)V.rho)[id] = (U)rho0;
}

// Pre-collision f(x, t) for diagnostics, as double SoA [19][nodes].
template <int P>
__global__ void k_read_f(const DomView* __restrict__ views, int dom, double* __restrict__ out) {
  using S = typename Store<P>::S;
  const DomView& V = views[dom];
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= V.N) return;
  const uint64_t t = V.tstep[0];  // steps completed: the gather of step t
  const bool inplace = V.inplace != 0, odd = (t & 1ull) != 0;
  const S* src = (const S*)((!inplace && odd) ? V.fB : V.fA);
  const int nx = V.n[0], ny = V.n[1], nz = V.n[2];
  const int nd[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((int64_t)nx * ny))};
  for (int a = 0; a < 3; ++a)
    if (V.bc[a] && (nd[a] == 0 || nd[a] == V.n[a] - 1)) {
      for (int i = 0; i < kQ; ++i) out[(int64_t)i * V.N + id] = 0.0;
      return;
    }
  for (int i = 0; i < kQ; ++i) {
    int s[3] = {nd[0] - kEx[i], nd[1] - kEy[i], nd[2] - kEz[i]};
    bool wall = false;
    for (int a = 0; a < 3; ++a) {
      if (V.bc[a]) wall |= (comp(i, a) != 0) && (s[a] == 0 || s[a] == V.n[a] - 1);
      else s[a] = s[a] < 0 ? s[a] + V.n[a] : (s[a] >= V.n[a] ? s[a] - V.n[a] : s[a]);
    }
    const int64_t up = s[0] + nx * ((int64_t)s[1] + (int64_t)ny * s[2]);
    size_t sidx;
    const uint32_t un = (uint32_t)id, uu = (uint32_t)up, NN = (uint32_t)V.N;
    if (!inplace) sidx = wall ? fidx(true, opp_dir(i), un, NN) : fidx(true, i, uu, NN);
    else if (!odd) sidx = fidx(false, i, un, NN);
    else sidx = wall ? fidx(false, i, un, NN) : fidx(false, opp_dir(i), uu, NN);
    double v = (double)to_c(src[sidx]);
    if (V.ibb && t > 0 && !wall && i > 0 && (V.smap[(t - 1) & 1ull][up] & kSolidBits)) {
      // interpolated bounce-back: what the next gather will take for this
      // link (the value of a solid node, or of a node uncovered since, is
      // not defined)
      using C = typename Store<P>::C;
      const C fso = to_c(src[fidx(true, opp_dir(i), un, NN)]);
      v = (double)ibb_link<P, false>(V, t, un, nd[0], nd[1], nd[2], i,
                                     (int)(V.smap[(t - 1) & 1ull][up] & kSolidBits) - 1, fso,
                                     nullptr);
    }
    if (P != P64) v = v + weight<double>(i) * V.rho0;
    out[(int64_t)i * V.N + id] = v;
  }
  (void)nz;
}

}  // namespace rwmi
