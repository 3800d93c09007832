// Two-way coupled particles (Sec. 2.2, Eq. 4-11): one launch per fluid step
// advances every coupled particle from t to t+1 in nsub substeps, with the
// hydrodynamic force and torque the fluid step of t accumulated (in 2^-48
// fixed point) in DomView::dem_acc, and writes the poses, rotated control
// points and filter spheres that the fluid of t+1 and the walkers of t read.
//
// One block of 64 threads (one wave), thread p owns particle p.  A substep:
//   force  m g + m a cos(2 pi tau / T) d + F_h (Eq. 4, the oscillator's
//          drive of Eq. 37 along d), torque T_h;
//   pairs  for the candidate partners j in ascending order: the closest
//          points of the two inner bodies (sphero-metaballs: an inner level
//          set M = cin dilated by a sphere of radius R_s) from the Newton-
//          Raphson stationary point of M_i + M_j (Eq. 6-8), the overlap and
//          normal of the dilation spheres (Eq. 9), the linear spring-dashpot
//          normal force and the tangential spring capped by Coulomb friction
//          (Eq. 5); the pair is evaluated with the lower index first by both
//          of its threads, so both apply the same force with opposite signs;
//   walls  the inner body's point whose gradient is normal to the wall
//          plane, by Newton-Raphson (Eq. 10-11);
//   update symplectic Euler for v, c and the angular momentum L, then
//          w = R I_b^-1 R^T L and the quaternion q += dt/2 (0, w) q,
//          normalised; the rotated offsets of the control points.
// Every sum runs in the same order as a plain sequential implementation
// (partners ascending, then walls by axis and side), each double operation
// rounded once, so the trajectory is reproducible bit for bit.
#pragma once
#include "dev_common.h"

namespace rwmi {

// Per-particle state record (doubles): c[3], v[3], q[4], L[3], w[3], Fh[3],
// Th[3], mass, Ib[9] (the 32 a read-out returns), Ibinv[9], cin, rb.
constexpr int kDemState = 44;
enum DemField { kDc = 0, kDv = 3, kDq = 6, kDL = 10, kDw = 13, kDFh = 16, kDTh = 19, kDm = 22, kDIb = 23,
                kDIbinv = 32, kDcin = 41, kDrb = 42 };
// Control points of all particles held in LDS by the particle update.
constexpr int kDemMaxCtrl = 1024;
// Substeps per fluid step (the drive's cosines of a step are tabulated in LDS).
constexpr int kDemMaxSub = 1024;
// Candidate partners of a step: bounding spheres within this margin at the
// step's start.  Two particles that each move less than half of it over the
// step cannot come into contact unnoticed (counter kDemSkin counts the
// particle steps that moved farther).
constexpr double kDemMargin = 1.0;

struct DemArgs {
  int32_t nsub, coupling, pad0, pad1;
  double g[3], drive_amp, drive_period, drive_dir[3];
  double kn, kt, eta_n, eta_t, mu, Rs;
  double* state;                // [np][kDemState]
  double* xi;                   // [64][64][3] tangential springs, row p owned by thread p
  double* xiw;                  // [64][6][3] wall springs (axis, side)
  unsigned long long* xmask;    // [64] bit j of row p: spring (p, j) may be nonzero
  double* ctrlr[3];             // writable views of DomView::ctrlr / ctrlr_f
  float* ctrlr_f[3];
};

// Slot k of a three-slot pointer table, selected without indexing (a
// runtime index would force the caller's copy of the table to memory).
template <typename T>
__device__ __forceinline__ T* slot_ptr(T* const (&tab)[3], int k) {
  return k == 0 ? tab[0] : (k == 1 ? tab[1] : tab[2]);
}

struct DemLds {
  double cosv[kDemMaxSub];  // cos(2 pi tau_s / T) of the step's substeps
  double wu[3][2][3];       // wall velocities
  double c[kMaxParticles][3], v[kMaxParticles][3], w[kMaxParticles][3];
  double rb[kMaxParticles], cin[kMaxParticles];
  float cf[kMaxParticles][4];  // centre and bounding radius in float: the candidate prefilter
  int nc[kMaxParticles], c0[kMaxParticles];
  double b[kDemMaxCtrl][3];   // offsets at the current orientation
  double bb[kDemMaxCtrl][3];  // offsets in the body frame
  double k[kDemMaxCtrl];
  // the particles whose rotated offsets the substeps read (a contact
  // candidate or a wall within reach), their rotations and the list of their
  // control points (particle << 16 | point), rotated by all lanes together
  int need[kMaxParticles];
  unsigned long long nbr2[kMaxParticles];  // candidates found by the second wave
  double R[kMaxParticles][9];
  uint32_t work[kDemMaxCtrl];
  int nwork;
  double F[kMaxParticles][3];  // force of the substep, for the translation wave
};

// ---------------------------------------------------------------- metaball
__device__ __forceinline__ double dem_M(const DemLds& S, int p, const double x[3]) {
  double M = 0.0;
  const int c0 = S.c0[p];
  for (int i = 0; i < S.nc[p]; ++i) {
    const double* b = S.b[c0 + i];
    const double rx = x[0] - b[0], ry = x[1] - b[1], rz = x[2] - b[2];
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == 0.0) return INFINITY;
    M = M + S.k[c0 + i] / r2;
  }
  return M;
}

__device__ __forceinline__ void dem_grad(const DemLds& S, int p, const double x[3], double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  const int c0 = S.c0[p];
  for (int i = 0; i < S.nc[p]; ++i) {
    const double* b = S.b[c0 + i];
    const double r[3] = {x[0] - b[0], x[1] - b[1], x[2] - b[2]};
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double q = (-2.0 * S.k[c0 + i]) / (r2 * r2);
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] = g[a] + q * r[a];
  }
}

// Hessian of M: sum_i k_i (8 r r^T / |r|^6 - 2 I / |r|^4).
__device__ __forceinline__ void dem_hess(const DemLds& S, int p, const double x[3], double H[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) H[a][c] = 0.0;
  const int c0 = S.c0[p];
  for (int i = 0; i < S.nc[p]; ++i) {
    const double* b = S.b[c0 + i];
    const double r[3] = {x[0] - b[0], x[1] - b[1], x[2] - b[2]};
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double r4 = r2 * r2;
    const double k = S.k[c0 + i];
    const double a8 = (8.0 * k) / (r4 * r2), a2 = (2.0 * k) / r4;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) H[a][c] = H[a][c] + (a8 * (r[a] * r[c]) - (a == c ? a2 : 0.0));
  }
}

// Inverse of a 3x3 matrix by cofactors; false when singular.
__device__ __forceinline__ bool dem_inv3(const double A[3][3], double X[3][3]) {
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double det = (A[0][0] * c00 + A[0][1] * c01) + A[0][2] * c02;
  if (det == 0.0 || !isfinite(det)) return false;
  X[0][0] = c00 / det;
  X[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
  X[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
  X[1][0] = c01 / det;
  X[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
  X[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
  X[2][0] = c02 / det;
  X[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
  X[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
  return true;
}

// Newton step st = A^-1 r; false when A is singular or the step not finite.
__device__ __forceinline__ bool dem_newton(const double A[3][3], const double r[3], double st[3]) {
  double X[3][3];
  if (!dem_inv3(A, X)) return false;
#pragma unroll
  for (int a = 0; a < 3; ++a) st[a] = (X[a][0] * r[0] + X[a][1] * r[1]) + X[a][2] * r[2];
  return isfinite(st[0]) && isfinite(st[1]) && isfinite(st[2]);
}

// Eq. 8: the point of p's inner body (level cin) reached from x along the
// gradient, with q from a first-order expansion of the field g = M^(-1/2)
// (same level sets as M; r / sqrt(k) for one control point, which makes the
// point exact for a sphere).  False when x is inside the inner body.
__device__ __forceinline__ bool dem_inner_point(const DemLds& S, int p, const double x[3], double xc[3]) {
  const double M = dem_M(S, p, x);
  const double cin = S.cin[p];
  if (!(M < cin)) return false;
  double gm[3];
  dem_grad(S, p, x, gm);
  const double g = 1.0 / sqrt(M), gin = 1.0 / sqrt(cin);
  const double s = -0.5 * (g / M);
  const double gg[3] = {s * gm[0], s * gm[1], s * gm[2]};
  const double n2 = (gg[0] * gg[0] + gg[1] * gg[1]) + gg[2] * gg[2];
  if (!(n2 > 0.0)) return false;
  const double q = (gin - g) / n2;
#pragma unroll
  for (int a = 0; a < 3; ++a) xc[a] = x[a] + q * gg[a];
  return true;
}

// Lattice extents and boundary kinds, held in registers by the particle
// update (a global view would be reloaded after every store it cannot rule
// out aliasing).
struct DemGeom {
  int n[3], bc[3];
};

// Minimum image of the displacement c_j - c_i on periodic axes.  Within a
// quarter period the image shift floor(dc / L + 0.5) is 0 (the quotient
// rounds into (-0.25, 0.25) at worst to +-0.25), and dc - L * 0 is dc bit for
// bit, so the division is skipped there.
__device__ __forceinline__ void dem_disp(const DemGeom& V, const double ci[3], const double cj[3], double dc[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dc[a] = cj[a] - ci[a];
    if (!V.bc[a]) {
      const double L = (double)V.n[a];
      if (!(fabs(dc[a]) < 0.25 * L)) dc[a] = dc[a] - L * floor(dc[a] / L + 0.5);
    }
  }
}


// Contact of particles i < j (Eq. 6-9).  True with the contact point as an
// offset from c_i, the normal from i's inner point to j's and the overlap.
__device__ __forceinline__ bool dem_contact_pair(const DemGeom& V, const DemArgs& A, const DemLds& S, int i, int j,
                                                 double xcp[3], double n[3], double& delta) {
  double dc[3];
  dem_disp(V, S.c[i], S.c[j], dc);
  const double r2 = dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2];
  const double rr = S.rb[i] + S.rb[j];
  if (!(r2 < rr * rr)) return false;
  double x[3] = {0.5 * dc[0], 0.5 * dc[1], 0.5 * dc[2]};
  for (int it = 0; it < 40; ++it) {
    const double xj[3] = {x[0] - dc[0], x[1] - dc[1], x[2] - dc[2]};
    double gi[3], gj[3], Hi[3][3], Hj[3][3], H[3][3], g[3], st[3];
    dem_grad(S, i, x, gi);
    dem_grad(S, j, xj, gj);
    dem_hess(S, i, x, Hi);
    dem_hess(S, j, xj, Hj);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      g[a] = gi[a] + gj[a];
#pragma unroll
      for (int c = 0; c < 3; ++c) H[a][c] = Hi[a][c] + Hj[a][c];
    }
    if (!dem_newton(H, g, st)) return false;
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = x[a] - st[a];
    const double sn = sqrt(st[0] * st[0] + st[1] * st[1] + st[2] * st[2]);
    if (sn < 1e-12) break;
  }
  const double xj[3] = {x[0] - dc[0], x[1] - dc[1], x[2] - dc[2]};
  double x0[3], x1[3], dd[3];
  if (!dem_inner_point(S, i, x, x0)) return false;
  if (!dem_inner_point(S, j, xj, x1)) return false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x1[a] = x1[a] + dc[a];
    dd[a] = x1[a] - x0[a];
  }
  const double dist = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  const double del = (A.Rs + A.Rs) - dist;
  if (!(del > 0.0) || !(dist > 0.0)) return false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    n[a] = dd[a] / dist;
    xcp[a] = x0[a] + (A.Rs - 0.5 * del) * n[a];
  }
  delta = del;
  return true;
}

// Contact of particle i with the wall plane of axis ax, side `side` (Eq.
// 10-11); the planes sit at 1 and n - 1 (halfway between the wall node and
// the first fluid node).  n points from the particle to the wall.
__device__ __forceinline__ bool dem_contact_wall(const DemGeom& V, const DemArgs& A, const DemLds& S, int i, int ax,
                                                 int side, double xcp[3], double n[3], double& delta) {
  const double* ci = S.c[i];
  const double plane = side ? (double)(V.n[ax] - 1) : 1.0;
  const double gap = side ? plane - ci[ax] : ci[ax] - plane;
  if (!(gap < S.rb[i] + A.Rs)) return false;
  const int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
  const double dir = side ? 1.0 : -1.0;
  const double cin = S.cin[i];
  double x[3] = {0.0, 0.0, 0.0};
  // start: the inner surface on the ray from the centre towards the wall
  double lo = 0.0, hi = S.rb[i];
  for (int it = 0; it < 60; ++it) {
    const double m = 0.5 * (lo + hi);
    double y[3] = {0.0, 0.0, 0.0};
    y[ax] = dir * m;
    if (dem_M(S, i, y) >= cin) lo = m;
    else hi = m;
  }
  x[ax] = dir * lo;
  for (int it = 0; it < 40; ++it) {
    double g[3], H[3][3], J[3][3], r[3], st[3];
    dem_grad(S, i, x, g);
    dem_hess(S, i, x, H);
    const double M = dem_M(S, i, x);
    r[0] = g[t1];
    r[1] = g[t2];
    r[2] = M - cin;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      J[0][c] = H[t1][c];
      J[1][c] = H[t2][c];
      J[2][c] = g[c];
    }
    if (!dem_newton(J, r, st)) return false;
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = x[a] - st[a];
    const double sn = sqrt(st[0] * st[0] + st[1] * st[1] + st[2] * st[2]);
    if (sn < 1e-12) break;
  }
  const double dist = side ? plane - (ci[ax] + x[ax]) : (ci[ax] + x[ax]) - plane;
  const double del = A.Rs - dist;
  if (!(del > 0.0)) return false;
#pragma unroll
  for (int a = 0; a < 3; ++a) n[a] = 0.0;
  n[ax] = dir;
#pragma unroll
  for (int a = 0; a < 3; ++a) xcp[a] = x[a] + (A.Rs - 0.5 * del) * n[a];
  delta = del;
  return true;
}

__device__ __forceinline__ void dem_cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Eq. 5 on body B from body A: normal n (A to B), overlap delta, relative
// velocity vr = v_B - v_A at the contact point, tangential spring xi
// (updated).  Normal force k_n delta minus the dashpot, never pulling;
// tangential -k_t xi - eta_t v_t, capped at mu F_n (the spring then set to
// what the capped force needs).
__device__ __forceinline__ void dem_contact_force(const DemArgs& A, const double n[3], double delta,
                                                  const double vr[3], double dt, double xi[3], double F[3]) {
  const double vn = (vr[0] * n[0] + vr[1] * n[1]) + vr[2] * n[2];
  double Fn = A.kn * delta - A.eta_n * vn;
  if (Fn < 0.0) Fn = 0.0;
  double vt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) vt[a] = vr[a] - vn * n[a];
#pragma unroll
  for (int a = 0; a < 3; ++a) xi[a] = xi[a] + vt[a] * dt;
  const double xn = (xi[0] * n[0] + xi[1] * n[1]) + xi[2] * n[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) xi[a] = xi[a] - xn * n[a];
  double Ft[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) Ft[a] = -(A.kt * xi[a]) - A.eta_t * vt[a];
  const double ft = sqrt((Ft[0] * Ft[0] + Ft[1] * Ft[1]) + Ft[2] * Ft[2]);
  const double cap = A.mu * Fn;
  if (ft > cap) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Ft[a] = Ft[a] * (cap / ft);
      xi[a] = A.kt > 0.0 ? -(Ft[a] + A.eta_t * vt[a]) / A.kt : 0.0;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] = Fn * n[a] + Ft[a];
}

// Rotation matrix of the unit quaternion (w, x, y, z).
__device__ __forceinline__ void dem_quat_R(const double q[4], double R[3][3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1.0 - 2.0 * (y * y + z * z);
  R[0][1] = 2.0 * (x * y - w * z);
  R[0][2] = 2.0 * (x * z + w * y);
  R[1][0] = 2.0 * (x * y + w * z);
  R[1][1] = 1.0 - 2.0 * (x * x + z * z);
  R[1][2] = 2.0 * (y * z - w * x);
  R[2][0] = 2.0 * (x * z - w * y);
  R[2][1] = 2.0 * (y * z + w * x);
  R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

// w = R I_b^-1 R^T L.
__device__ __forceinline__ void dem_omega(const double R[3][3], const double* Ibinv, const double L[3], double w[3]) {
  double y[3], z[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) y[a] = (R[0][a] * L[0] + R[1][a] * L[1]) + R[2][a] * L[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) z[a] = (Ibinv[3 * a] * y[0] + Ibinv[3 * a + 1] * y[1]) + Ibinv[3 * a + 2] * y[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) w[a] = (R[a][0] * z[0] + R[a][1] * z[1]) + R[a][2] * z[2];
}

// One substep of the rotation: L += T dt, w = R I_b^-1 R^T L, q += dt/2
// (0, w) q normalised, and R of the new q.
__device__ __forceinline__ void dem_rotate(const double T[3], double dt, const double* Ibinv, double L[3], double w[3],
                                           double q[4], double Rc[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) L[a] = L[a] + T[a] * dt;
  dem_omega(Rc, Ibinv, L, w);
  const double w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3];
  const double hw[3] = {0.5 * dt * w[0], 0.5 * dt * w[1], 0.5 * dt * w[2]};
  const double n0 = w0 - ((hw[0] * w1 + hw[1] * w2) + hw[2] * w3);
  const double n1 = w1 + ((hw[0] * w0 + hw[1] * w3) - hw[2] * w2);
  const double n2 = w2 + ((hw[1] * w0 + hw[2] * w1) - hw[0] * w3);
  const double n3 = w3 + ((hw[2] * w0 + hw[0] * w2) - hw[1] * w1);
  const double nn = sqrt(((n0 * n0 + n1 * n1) + n2 * n2) + n3 * n3);
  q[0] = n0 / nn;
  q[1] = n1 / nn;
  q[2] = n2 / nn;
  q[3] = n3 / nn;
  dem_quat_R(q, Rc);
}

// One substep of the translation (symplectic Euler) with the periodic wrap.
__device__ __forceinline__ void dem_translate(const DemGeom& G, const double F[3], double mass, double dt, double v[3],
                                              double c[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    v[a] = v[a] + (F[a] / mass) * dt;
    c[a] = c[a] + v[a] * dt;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (!G.bc[a]) {
      const double Ln = (double)G.n[a];
      c[a] = c[a] - Ln * floor(c[a] / Ln);
    }
}

// The particle update of step t = tstep + j (t -> t+1).  Launch: one block
// of 64 threads per domain.
// Two waves of 64 lanes, lane p of each for particle p: the first finds the
// contacts and forces, integrates the rotation and writes the results; the
// second integrates the translation (v, c), which depends on the rotation
// of no substep, so the two chains of a substep run side by side.
__device__ __forceinline__ void dem_block(const DomView& V, const DemArgs& A, uint64_t t, DemLds& S) {
  const int tid = threadIdx.x;
  const bool main = tid < kMaxParticles;  // contacts, rotation, results
  const int p = tid & (kMaxParticles - 1);
  const int np = V.np;
  const unsigned long long dmask = V.dem_mask;
  DemGeom G;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    G.n[a] = V.n[a];
    G.bc[a] = V.bc[a];
  }
  const bool live = p < np;
  const bool cp = live && ((dmask >> p) & 1ull);
  // the drive of every substep of the step, in parallel
  const double dt = 1.0 / (double)A.nsub;
  for (int s = tid; s < A.nsub; s += blockDim.x) {
    const double tau = (double)t + (double)s * dt;
    double ph = tau / A.drive_period;
    ph = ph - floor(ph);
    double sn, cs;
    sincos_turns(ph, sn, cs);
    S.cosv[s] = cs;
  }
  if (tid < 18) S.wu[tid / 6][(tid / 3) & 1][tid % 3] = V.wu[tid / 6][(tid / 3) & 1][tid % 3];
  if (main) S.need[p] = 0;
  const DevParticle* P = live ? V.parts + p : nullptr;
  double* st = live ? A.state + (size_t)kDemState * p : nullptr;
  double c[3] = {0, 0, 0}, v[3] = {0, 0, 0}, q[4] = {1, 0, 0, 0}, L[3] = {0, 0, 0}, w[3] = {0, 0, 0};
  double Fh[3] = {0, 0, 0}, Th[3] = {0, 0, 0}, mass = 1.0, Ibinv[9];
  const int sl = pose_slot(t);  // slot of the control points at P(t)
  if (cp && !main) {  // the translation wave
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = st[kDc + a];
      v[a] = st[kDv + a];
    }
    mass = st[kDm];
  }
  if (cp && main) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = st[kDc + a];
      v[a] = st[kDv + a];
      L[a] = st[kDL + a];
      w[a] = st[kDw + a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) q[a] = st[kDq + a];
#pragma unroll
    for (int a = 0; a < 9; ++a) Ibinv[a] = st[kDIbinv + a];
    mass = st[kDm];
    unsigned long long* acc = V.dem_acc + 6 * p;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Fh[a] = A.coupling ? (double)(long long)acc[a] / kForceFix : 0.0;
      Th[a] = A.coupling ? (double)(long long)acc[3 + a] / kForceFix : 0.0;
      S.F[p][a] = Fh[a];  // for the second wave if no substep has contacts
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = 0ull;  // for the next fluid step
  }
  if (np > 0) {  // the control points of all particles (contiguous), all threads
    const DevParticle* last = V.parts + (np - 1);
    const int nct = last->ctrl0 + last->nc;
    const double* src = slot_ptr(A.ctrlr, sl);
    for (int e = tid; e < nct; e += blockDim.x) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        S.b[e][a] = src[4 * e + a];
        S.bb[e][a] = V.ctrl[4 * e + a];
      }
      S.k[e] = src[4 * e + 3];
    }
  }
  if (live && main) {
    S.nc[p] = P->nc;
    S.c0[p] = P->ctrl0;
    S.rb[p] = cp ? st[kDrb] : P->rb;
    S.cin[p] = cp ? st[kDcin] : 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      S.c[p][a] = c[a];
      S.v[p][a] = v[a];
      S.w[p][a] = w[a];
      S.cf[p][a] = (float)c[a];
    }
    S.cf[p][3] = (float)S.rb[p];
  }
  __syncthreads();
  // candidate partners of the step; the springs of every other pair are zero
  // (xnz: the partners whose spring may be nonzero)
  unsigned long long nbr = 0ull, xnz = 0ull;
  const double cstart[3] = {c[0], c[1], c[2]};
  // The two waves share the test: lane p of the first tries the particles
  // below half of np, lane p of the second (which holds the same centre)
  // the others.
  // Each pair is first measured in float.  With every lattice edge at most
  // 4096 the float distance of the centres' nearest images is within about
  // 1.2e-3 of the exact one (positions rounded to 2^-12, their differences
  // and squares to 2^-24 relative), and near half a period both images are
  // about as long; so a float gap more than 0.01 from the candidate
  // threshold decides the FP64 test's outcome, and only pairs closer to the
  // threshold (or on larger lattices) take that test.
  if (cp) {
    const int half = (np + 1) >> 1;
    const int j0 = main ? 0 : half, j1 = main ? half : np;
    const double rbp = S.rb[p];
    const float cpf[3] = {S.cf[p][0], S.cf[p][1], S.cf[p][2]};
    const float rbpf = S.cf[p][3];
    const float Lf[3] = {(float)G.n[0], (float)G.n[1], (float)G.n[2]};
    const float band = (G.n[0] <= 4096 && G.n[1] <= 4096 && G.n[2] <= 4096) ? 0.01f : 3.4e38f;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
      float d2 = 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float d = S.cf[j][a] - cpf[a];
        if (!G.bc[a]) {
          d = fabsf(d);
          d = d > 0.5f * Lf[a] ? Lf[a] - d : d;
        }
        d2 += d * d;
      }
      const float gap = __builtin_sqrtf(d2) - ((rbpf + S.cf[j][3]) + (float)kDemMargin);
      bool cand;
      if (gap > band) cand = false;
      else if (gap < -band) cand = true;
      else {
        double dc[3];
        dem_disp(G, c, S.c[j], dc);
        const double r2 = dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2];
        const double rr = (rbp + S.rb[j]) + kDemMargin;
        cand = r2 < rr * rr;
      }
      cand = cand && j != p && ((dmask >> j) & 1ull) != 0ull;
      nbr |= (unsigned long long)cand << j;
    }
    if (!main) S.nbr2[p] = nbr;
  }
  __syncthreads();
  if (cp && main) {
    nbr |= S.nbr2[p];
    // Only the springs the previous step may have left nonzero (a superset
    // kept in xmask) are read: every other one is zero.  A nonzero spring
    // of a candidate is carried over, one of any other pair cleared.
    unsigned long long held = A.xmask[p];
    while (held) {
      const int j = __ffsll((long long)held) - 1;
      held &= held - 1ull;
      double* x = A.xi + ((size_t)p * kMaxParticles + j) * 3;
      if (!(x[0] != 0.0 || x[1] != 0.0 || x[2] != 0.0)) continue;
      if ((nbr >> j) & 1ull) xnz |= 1ull << j;
      else x[0] = x[1] = x[2] = 0.0;
    }
  }
  unsigned wnz = 0u;  // walls whose spring may be nonzero (bit 2 axis + side)
  if (cp && main)
    for (int k = 0; k < 6; ++k) {
      if (!G.bc[k >> 1]) continue;  // no wall plane: never written, zero
      const double* x = A.xiw + ((size_t)p * 6 + k) * 3;
      if (x[0] != 0.0 || x[1] != 0.0 || x[2] != 0.0) wnz |= 1u << k;
    }
  // Rotated offsets are read only by contacts: a particle with a candidate
  // partner or a wall plane within reach (bounding radius + R_s + the
  // candidates' margin) at the start of the step has them rotated every
  // substep, together with its partners; the others only once, after the
  // last substep (the same values: a rotation depends on q alone).
  if (cp && main) {
    bool wall = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
      if (G.bc[ax]) {
        const double reach = (S.rb[p] + A.Rs) + kDemMargin;
        wall = wall || (c[ax] - 1.0 < reach) || ((double)(G.n[ax] - 1) - c[ax] < reach);
      }
    if (nbr || wall) {
      S.need[p] = 1;
      unsigned long long bits = nbr;
      while (bits) {
        const int j = __ffsll((long long)bits) - 1;
        bits &= bits - 1ull;
        S.need[j] = 1;
      }
    }
  }
  __syncthreads();
  const unsigned long long needm = __ballot(main && S.need[p] != 0);  // the first wave's flags
  if (tid == 0) {
    int k = 0;
    unsigned long long bits = needm;
    while (bits) {
      const int i = __ffsll((long long)bits) - 1;
      bits &= bits - 1ull;
      for (int m = 0; m < S.nc[i]; ++m) S.work[k++] = ((uint32_t)i << 16) | (uint32_t)(S.c0[i] + m);
    }
    S.nwork = k;
  }
  __syncthreads();
  const int nwork = S.nwork;
  const bool need = live && S.need[p] != 0;
  double Rc[3][3];  // rotation of the current q
  dem_quat_R(q, Rc);
  if (nwork == 0 && !G.bc[0] && !G.bc[1] && !G.bc[2]) {
    // No particle has a contact candidate and there are no wall planes: no
    // substep reads another particle's state, so each wave runs its chain
    // of substeps without barriers.  The second wave forms each substep's
    // force itself, from the terms the first wave would have summed (F_h
    // it left in S.F); contacts would have added to them, and there are
    // none.  The operations are those of the loop below, in its order.
    if (cp && !main) {
      const double fh[3] = {S.F[p][0], S.F[p][1], S.F[p][2]};
      for (int s = 0; s < A.nsub; ++s) {
        const double cs = S.cosv[s];
        double F[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) F[a] = (mass * A.g[a] + mass * ((A.drive_amp * cs) * A.drive_dir[a])) + fh[a];
        dem_translate(G, F, mass, dt, v, c);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        S.c[p][a] = c[a];
        S.v[p][a] = v[a];
      }
    }
    if (cp && main)
      for (int s = 0; s < A.nsub; ++s) dem_rotate(Th, dt, Ibinv, L, w, q, Rc);
    __syncthreads();  // the final centres and velocities are visible
  } else {
    double cs_next = S.cosv[0];  // the drive of the next substep, read ahead
    for (int s = 0; s < A.nsub; ++s) {
      double F[3], T[3];
      const double cs = cs_next;
      if (s + 1 < A.nsub) cs_next = S.cosv[s + 1];
      if (cp && main) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          F[a] = (mass * A.g[a] + mass * ((A.drive_amp * cs) * A.drive_dir[a])) + Fh[a];
          T[a] = Th[a];
        }
        unsigned long long bits = nbr;
        while (bits) {
          const int j = __ffsll((long long)bits) - 1;
          bits &= bits - 1ull;
          const int i0 = p < j ? p : j, i1 = p < j ? j : p;
          double* xi = A.xi + ((size_t)p * kMaxParticles + j) * 3;
          double xcp[3], n[3], del;
          if (!dem_contact_pair(G, A, S, i0, i1, xcp, n, del)) {
            if ((xnz >> j) & 1ull) {
              xi[0] = xi[1] = xi[2] = 0.0;
              xnz &= ~(1ull << j);
            }
            continue;
          }
          double dc[3], rj[3], wa[3], wb[3], vr[3], Fc[3];
          dem_disp(G, S.c[i0], S.c[i1], dc);
#pragma unroll
          for (int a = 0; a < 3; ++a) rj[a] = xcp[a] - dc[a];
          dem_cross(S.w[i0], xcp, wa);
          dem_cross(S.w[i1], rj, wb);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double va = S.v[i0][a] + wa[a];
            const double vb = S.v[i1][a] + wb[a];
            vr[a] = vb - va;
          }
          double xv[3] = {0.0, 0.0, 0.0};
          if ((xnz >> j) & 1ull) {
            xv[0] = xi[0];
            xv[1] = xi[1];
            xv[2] = xi[2];
          }
          dem_contact_force(A, n, del, vr, dt, xv, Fc);
          xi[0] = xv[0];
          xi[1] = xv[1];
          xi[2] = xv[2];
          xnz |= 1ull << j;
          double tq[3];
          if (p == i1) {
            dem_cross(rj, Fc, tq);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              F[a] = F[a] + Fc[a];
              T[a] = T[a] + tq[a];
            }
          } else {
            const double mF[3] = {-Fc[0], -Fc[1], -Fc[2]};
            dem_cross(xcp, mF, tq);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              F[a] = F[a] + mF[a];
              T[a] = T[a] + tq[a];
            }
          }
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          if (!G.bc[ax]) continue;
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int k = 2 * ax + side;
            double* xi = A.xiw + ((size_t)p * 6 + k) * 3;
            double xcp[3], n[3], del;
            if (!dem_contact_wall(G, A, S, p, ax, side, xcp, n, del)) {
              if ((wnz >> k) & 1u) {
                xi[0] = xi[1] = xi[2] = 0.0;
                wnz &= ~(1u << k);
              }
              continue;
            }
            double wa[3], vr[3], Fc[3];
            dem_cross(S.w[p], xcp, wa);
#pragma unroll
            for (int a = 0; a < 3; ++a) vr[a] = S.wu[ax][side][a] - (S.v[p][a] + wa[a]);
            double xv[3] = {0.0, 0.0, 0.0};
            if ((wnz >> k) & 1u) {
              xv[0] = xi[0];
              xv[1] = xi[1];
              xv[2] = xi[2];
            }
            dem_contact_force(A, n, del, vr, dt, xv, Fc);
            xi[0] = xv[0];
            xi[1] = xv[1];
            xi[2] = xv[2];
            wnz |= 1u << k;
            const double mF[3] = {-Fc[0], -Fc[1], -Fc[2]};
            double tq[3];
            dem_cross(xcp, mF, tq);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              F[a] = F[a] + mF[a];
              T[a] = T[a] + tq[a];
            }
          }
        }
      }
      if (cp && main)
#pragma unroll
        for (int a = 0; a < 3; ++a) S.F[p][a] = F[a];
      __syncthreads();  // every contact of the substep has read the shared state
      if (cp && !main) {  // translation
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          v[a] = v[a] + (S.F[p][a] / mass) * dt;
          c[a] = c[a] + v[a] * dt;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
          if (!G.bc[a]) {
            const double Ln = (double)G.n[a];
            c[a] = c[a] - Ln * floor(c[a] / Ln);
          }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          S.c[p][a] = c[a];
          S.v[p][a] = v[a];
        }
      }
      if (cp && main) {  // rotation
#pragma unroll
        for (int a = 0; a < 3; ++a) L[a] = L[a] + T[a] * dt;
        dem_omega(Rc, Ibinv, L, w);
        const double w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3];
        const double hw[3] = {0.5 * dt * w[0], 0.5 * dt * w[1], 0.5 * dt * w[2]};
        const double n0 = w0 - ((hw[0] * w1 + hw[1] * w2) + hw[2] * w3);
        const double n1 = w1 + ((hw[0] * w0 + hw[1] * w3) - hw[2] * w2);
        const double n2 = w2 + ((hw[1] * w0 + hw[2] * w1) - hw[0] * w3);
        const double n3 = w3 + ((hw[2] * w0 + hw[0] * w2) - hw[1] * w1);
        const double nn = sqrt(((n0 * n0 + n1 * n1) + n2 * n2) + n3 * n3);
        q[0] = n0 / nn;
        q[1] = n1 / nn;
        q[2] = n2 / nn;
        q[3] = n3 / nn;
        dem_quat_R(q, Rc);
        if (need)
#pragma unroll
          for (int a = 0; a < 9; ++a) S.R[p][a] = Rc[a / 3][a % 3];
#pragma unroll
        for (int a = 0; a < 3; ++a) S.w[p][a] = w[a];
      }
      if (nwork) {
        __syncthreads();  // the new rotations are visible
        // offsets at the new orientation from the body-frame control points
        for (int k = tid; k < nwork; k += blockDim.x) {
          const uint32_t e = S.work[k];
          const double* R = S.R[e >> 16];
          const int i = (int)(e & 0xFFFFu);
          const double* bb = S.bb[i];
#pragma unroll
          for (int a = 0; a < 3; ++a) S.b[i][a] = (R[3 * a] * bb[0] + R[3 * a + 1] * bb[1]) + R[3 * a + 2] * bb[2];
        }
      }
      __syncthreads();  // the new state is visible to every contact of the next substep
    }
  }
  if (!main) return;
  if (cp) A.xmask[p] = xnz;  // the springs this step may leave nonzero
  if (cp)  // the translation wave's final centre and velocity
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = S.c[p][a];
      v[a] = S.v[p][a];
    }
  if (cp && !need) {  // offsets at the final orientation
    const int c0 = S.c0[p];
    for (int i = 0; i < S.nc[p]; ++i) {
      const double* bb = S.bb[c0 + i];
#pragma unroll
      for (int a = 0; a < 3; ++a) S.b[c0 + i][a] = (Rc[a][0] * bb[0] + Rc[a][1] * bb[1]) + Rc[a][2] * bb[2];
    }
  }
  if (!live) return;
  // results: state, pose tables of P(t+1), filter sphere, control points
  const int sn = pose_slot(t + 1);
  double pc[3], pv[3], pw[3] = {0.0, 0.0, 0.0};
  if (cp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      st[kDc + a] = c[a];
      st[kDv + a] = v[a];
      st[kDL + a] = L[a];
      st[kDw + a] = w[a];
      st[kDFh + a] = Fh[a];
      st[kDTh + a] = Th[a];
      pc[a] = c[a];
      pv[a] = v[a];
      pw[a] = w[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) st[kDq + a] = q[a];
    double d2 = 0.0;
    double dc[3];
    dem_disp(G, cstart, c, dc);
#pragma unroll
    for (int a = 0; a < 3; ++a) d2 = d2 + dc[a] * dc[a];
    if (d2 > 0.25 * kDemMargin * kDemMargin) counter_add(V.counters + kDemSkin, 1ull);
    const int c0 = S.c0[p];
    double* dst = slot_ptr(A.ctrlr, sn);
    float* dstf = slot_ptr(A.ctrlr_f, sn);
    for (int i = 0; i < S.nc[p]; ++i) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        dst[4 * (c0 + i) + a] = S.b[c0 + i][a];
        dstf[4 * (c0 + i) + a] = (float)S.b[c0 + i][a];
      }
      dst[4 * (c0 + i) + 3] = S.k[c0 + i];
      dstf[4 * (c0 + i) + 3] = (float)S.k[c0 + i];
    }
  } else {
    particle_pose(*P, t + 1, pc, pv);
  }
  double* pn = V.pose[sl] + kPoseRec * (np + p);  // walkers of step t: P(t+1)
  double* pf = V.pose[sn] + kPoseRec * p;         // fluid of step t+1: P(t+1)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    pn[a] = pc[a];
    pn[3 + a] = pv[a];
    pn[6 + a] = pw[a];
    pf[a] = pc[a];
    pf[3 + a] = pv[a];
    pf[6 + a] = pw[a];
  }
  using F4 = float __attribute__((ext_vector_type(4)));
  const float rs = (float)P->maskr + kSphereMargin;
  const F4 sp = {(float)pc[0], (float)pc[1], (float)pc[2], rs * rs};
  *gp((F4*)V.sph[sl] + p) = sp;
}

// Pose tables of step t from the state (the set-up of the coupling, or a
// change of a particle's motion): P(t) for the fluid of t (slot t mod 3),
// the control points of the coupled particles at their orientation.
__device__ __forceinline__ void dem_tables(const DomView& V, const DemArgs& A, uint64_t t) {
  const int p = threadIdx.x;
  if (p >= V.np) return;
  const int sl = pose_slot(t);
  const bool cp = (V.dem_mask >> p) & 1ull;
  double pc[3], pv[3], pw[3] = {0.0, 0.0, 0.0};
  const DevParticle* P = V.parts + p;
  if (cp) {
    const double* st = A.state + (size_t)kDemState * p;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pc[a] = st[kDc + a];
      pv[a] = st[kDv + a];
      pw[a] = st[kDw + a];
    }
    double R[3][3];
    const double q[4] = {st[kDq], st[kDq + 1], st[kDq + 2], st[kDq + 3]};
    dem_quat_R(q, R);
    const int c0 = P->ctrl0;
    double* dst = slot_ptr(A.ctrlr, sl);
    float* dstf = slot_ptr(A.ctrlr_f, sl);
    for (int i = 0; i < P->nc; ++i) {
      const double* bb = V.ctrl + 4 * (c0 + i);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double x = (R[a][0] * bb[0] + R[a][1] * bb[1]) + R[a][2] * bb[2];
        dst[4 * (c0 + i) + a] = x;
        dstf[4 * (c0 + i) + a] = (float)x;
      }
      dst[4 * (c0 + i) + 3] = bb[3];
      dstf[4 * (c0 + i) + 3] = (float)bb[3];
    }
  } else {
    particle_pose(*P, t, pc, pv);
  }
  double* pf = V.pose[sl] + kPoseRec * p;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    pf[a] = pc[a];
    pf[3 + a] = pv[a];
    pf[6 + a] = pw[a];
  }
}

}  // namespace rwmi
