/*
 * FP64 CPU oracle for one coupled RW-MI-DELBM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path: both are written independently from the paper
 * (arXiv 2308.05007) and from the readings of it recorded in the design notes.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 * (no FMA contraction, no fast-math, IEEE double on x86-64 SSE2).
 *
 * What is computed (paper sections in brackets):
 *   fluid    : D3Q19 BGK lattice Boltzmann (Sec. 2.3, Eq. 12-15), collide then
 *              stream; the moving-wall term of the bounce-back rule has the
 *              form of Eq. 23 (with C = 1).  Particles enter through the
 *              partially saturated cell method (named in Sec. 1) with the
 *              Noble-Torczynski weighting; a uniform body force enters by the
 *              Guo forcing scheme.  Neither PSM's formula nor the forcing is
 *              printed in the paper: both are readings.
 *   particles: metaball function and gradient (Eq. 3, Eq. 17), prescribed
 *              rigid motion (the oscillator of Sec. 4, Eq. 37 read as a
 *              displacement sinusoid), rigid surface velocity (Sec. 2.4.3);
 *              or two-way coupled particles: Newton-Euler motion (Eq. 4)
 *              under gravity, the drive of Eq. 37, the hydrodynamic force
 *              and torque of the PSM momentum exchange and the contacts of
 *              Eq. 5-11 (sphero-metaball pairs and walls).
 *   solute   : random-walk update (Eq. 2) with trilinear velocity
 *              interpolation (Sec. 2.4.1), walker/particle types I-IV
 *              (Sec. 2.4.2), binary search for the intersection (Algorithm 1),
 *              specular reflection (Algorithm 2, Eq. 18-22), refill of type II
 *              walkers and return-to-origin in narrow gaps (Sec. 2.4.2),
 *              concentration as a node count (Eq. 16).
 *   random   : Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
 *              seed, counter (walker, step, purpose, 0); Box-Muller normals
 *              built from our own LN and SINCOS2PI that use only +,-,*,/,sqrt
 *              so that any IEEE machine reproduces them bit for bit.
 *   reports  : occupancy n_s (Eq. 16), FP64 moments feeding Eq. 38-40.
 *
 * Every sum is taken left to right in the order stated next to it.
 *
 * Pins (tests/test_oracle_*.py and tests/test_dispersion.py check these
 * against mathematics other than this code):
 *   equilibrium     lattice isotropy sums; mass, momentum and second moment
 *                   of f^eq (textbook invariants)
 *   collision       mass conserved, momentum grows by exactly F per node and
 *                   step, tau = 1 relaxes to f^eq, a rest state stays at rest
 *                   bitwise; PSM: eps = 0 ignores the solid velocity, a fully
 *                   solid node relaxes to u_s, momentum exchange per node, and
 *                   direction by direction f^eq(u) + g maps to the closed-form
 *                   blend (1-B) f^eq(u) + B f^eq(u_s) + (1-B)(1-1/tau) g + B g_opp
 *   streaming       pull equals a separately written push (brute force);
 *                   Poiseuille at the exact tau (closed form), curvature at any
 *                   tau, Couette linear profile
 *   metaball        one control point is a sphere of radius sqrt(k) (with
 *                   Table 1's sphere: projected area 78.54 at k = 25); two equal
 *                   points give the mid-plane ring; gradient vs central
 *                   differences; bounding-radius lemma; minimum image
 *   solid fraction  one control point: eps = 1/2 + (sqrt(k) - r) exactly, the
 *                   sphere volume V + pi R / 3 by quadrature.  Two control
 *                   points (equal and unequal weights): 1/2 + d matches the
 *                   exact signed distance to the surface within the
 *                   second-order bound of a first-order estimate, and eps is
 *                   exactly 0 or 1 beyond the ramp.
 *   Algorithm 1, 2  crossing of a one-point sphere vs the quadratic root;
 *                   iteration cap; |t_r| = |t_i|, t_r.n = -t_i.n, specular on
 *                   a sphere
 *   random          Philox words vs rocRAND's philox4x32_10 (library
 *                   cross-check); LN and SINCOS2PI vs long-double libm;
 *                   normals: moments, KS, bound
 *   walkers         free-space MSD = 6 D t, also with steps of several
 *                   periods (image counts); plume drift and spread (Eq. 31,
 *                   34); walls confine and keep a uniform density; reflection
 *                   keeps walkers out of a static particle; count conserved;
 *                   a non-finite step and a wall reflection still outside the
 *                   fluid range return the walker (closed form per walker)
 *   interpolation   displacement at D = 0 equals the closed-form tensor
 *                   product of 1-D chords of a per-axis quadratic field, and
 *                   the Couette profile with the wall nodes' velocity
 *   moments         Poiseuille mean and momentum; fluid and particle averages
 *                   and solid volume of two spheres in a prescribed flow
 *   type II refill  the refilled walker lies outside every particle and near
 *                   the surface, count conserved; on a sphere the refill
 *                   point matches its closed form (radial exit, outer half
 *                   ball of radius sqrt(2D)) and is uniform in that half
 *                   ball.  How the point is chosen is a reading.
 *   dispersion fit  a linear variance series gives the closed-form K and
 *                   D_alpha; pure diffusion gives sigma^2 = 2 D t
 *   coupled         (tests/test_oracle_dem.py) mass and inertia of a sphere
 *   particles       (closed form) and of an asymmetric metaball (fine-grid
 *                   indicator integral); the body stays where it was given;
 *                   free fall and the drive as closed sums of symplectic
 *                   Euler; elastic and damped head-on collisions (momentum,
 *                   restitution of a linear spring-dashpot); static overlap
 *                   m g / k_n on a wall and of two stacked spheres (exact
 *                   closest points); sliding at mu g, then rolling at 5/7 v0;
 *                   angular momentum of an oblique frictional collision;
 *                   free precession of a symmetric body (first order);
 *                   fluid + particle momentum conserved; Stokes torque on a
 *                   spinning sphere within 10%; thread-count independent
 *                   force sums
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXP 64
#define ORC_NCNT 8

/* ---------------------------------------------------------------- D3Q19 */
/* Textbook D3Q19 (Qian, d'Humieres, Lallemand 1992); the paper names the
 * model (Sec. 2.3) but prints neither the velocities nor the weights.
 * Order: rest, the six axis directions (+x,-x,+y,-y,+z,-z), then the twelve
 * diagonals in opposite pairs.  c_s^2 = 1/3. */
static const int EV[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static double WT[19];

static int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

static void init_weights(void) {
  WT[0] = 1.0 / 3.0;
  for (int i = 1; i <= 6; i++) WT[i] = 1.0 / 18.0;
  for (int i = 7; i <= 18; i++) WT[i] = 1.0 / 36.0;
}

/* e_i . v summed over x, y, z; a zero component contributes nothing. */
static double edot(int i, const double v[3]) {
  double s = 0.0;
  for (int a = 0; a < 3; a++) {
    if (EV[i][a] == 1) s = s + v[a];
    else if (EV[i][a] == -1) s = s - v[a];
  }
  return s;
}

/* Eq. 13 with c_s^2 = 1/3:  w_i rho [1 + 3 eu + 4.5 eu^2 - 1.5 u.u]. */
static double feq(int i, double rho, const double u[3]) {
  double eu = edot(i, u);
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return (WT[i] * rho) * (((1.0 + 3.0 * eu) + 4.5 * (eu * eu)) - 1.5 * uu);
}

/* ------------------------------------------------------------ Philox */
/* Philox4x32-10 as published: ten rounds of the 4x32 S-box
 * (hi(M0 c0), lo(M0 c0), hi(M1 c2), lo(M1 c2)) mixed with the key, the key
 * bumped by the Weyl constants between rounds. */
static void philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* (r + 1/2) 2^-32: exact in double, strictly inside (0, 1). */
static double u01(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

/* Natural log of a positive normal double: u = m 2^e with m in (sqrt(1/2),
 * sqrt(2)], ln m = 2 atanh(s) = 2s (1 + s^2/3 + s^4/5 + ...), s = (m-1)/(m+1),
 * eleven terms (|s| < 0.1716, truncation below 1e-17), then e ln2 with ln2
 * split in a high part with trailing zeros and a low remainder. */
static double orc_ln(double u) {
  uint64_t bits;
  memcpy(&bits, &u, 8);
  int e = (int)((bits >> 52) & 0x7ff) - 1023;
  uint64_t mb = (bits & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL;
  double m;
  memcpy(&m, &mb, 8);
  if (m > 0x1.6a09e667f3bcdp+0) { /* sqrt(2) rounded */
    m = m * 0.5;
    e = e + 1;
  }
  double s = (m - 1.0) / (m + 1.0);
  double s2 = s * s;
  double p = 1.0 / 21.0;
  p = p * s2 + 1.0 / 19.0;
  p = p * s2 + 1.0 / 17.0;
  p = p * s2 + 1.0 / 15.0;
  p = p * s2 + 1.0 / 13.0;
  p = p * s2 + 1.0 / 11.0;
  p = p * s2 + 1.0 / 9.0;
  p = p * s2 + 1.0 / 7.0;
  p = p * s2 + 1.0 / 5.0;
  p = p * s2 + 1.0 / 3.0;
  double t = 2.0 * s;
  double lnm = t + (t * s2) * p;
  double de = (double)e;
  return de * 0x1.62e42feep-1 + (de * 0x1.a39ef35793c76p-33 + lnm);
}

/* Taylor polynomials of sin and cos on [0, pi/4]: degree 17 and 16. */
static double sin_poly(double x) {
  double x2 = x * x;
  double p = 1.0 / 355687428096000.0;
  p = p * x2 - 1.0 / 1307674368000.0;
  p = p * x2 + 1.0 / 6227020800.0;
  p = p * x2 - 1.0 / 39916800.0;
  p = p * x2 + 1.0 / 362880.0;
  p = p * x2 - 1.0 / 5040.0;
  p = p * x2 + 1.0 / 120.0;
  p = p * x2 - 1.0 / 6.0;
  return x + (x * x2) * p;
}
static double cos_poly(double x) {
  double x2 = x * x;
  double p = 1.0 / 20922789888000.0;
  p = p * x2 - 1.0 / 87178291200.0;
  p = p * x2 + 1.0 / 479001600.0;
  p = p * x2 - 1.0 / 3628800.0;
  p = p * x2 + 1.0 / 40320.0;
  p = p * x2 - 1.0 / 720.0;
  p = p * x2 + 1.0 / 24.0;
  p = p * x2 - 1.0 / 2.0;
  return 1.0 + x2 * p;
}

/* sin(2 pi u), cos(2 pi u) for u in [0, 1): exact quadrant split q = floor(4u),
 * f = 4u - q; reduce to [0, pi/4] by f -> 1 - f (both exact), then rotate by
 * q quarter turns. */
static void sincos2pi(double u, double* s, double* c) {
  double t4 = 4.0 * u;
  double qd = floor(t4);
  double f = t4 - qd;
  int q = (int)qd & 3;
  double s0, c0;
  if (f <= 0.5) {
    double x = f * 0x1.921fb54442d18p+0; /* pi/2 */
    s0 = sin_poly(x);
    c0 = cos_poly(x);
  } else {
    double x = (1.0 - f) * 0x1.921fb54442d18p+0;
    s0 = cos_poly(x);
    c0 = sin_poly(x);
  }
  switch (q) {
    case 0: *s = s0; *c = c0; break;
    case 1: *s = c0; *c = -s0; break;
    case 2: *s = -s0; *c = -c0; break;
    default: *s = -c0; *c = s0; break;
  }
}

/* Box-Muller on the four words of one Philox block: z0, z1 from (r0, r1),
 * z2 from (r2, r3).  The paper asks only for zero-mean unit-variance
 * Gaussian z (Eq. 2). */
static void normals3(const uint32_t r[4], double z[3]) {
  double R0 = sqrt(-2.0 * orc_ln(u01(r[0])));
  double s, c;
  sincos2pi(u01(r[1]), &s, &c);
  z[0] = R0 * c;
  z[1] = R0 * s;
  double R2 = sqrt(-2.0 * orc_ln(u01(r[2])));
  sincos2pi(u01(r[3]), &s, &c);
  z[2] = R2 * c;
}

/* ----------------------------------------------------------- domain */
typedef struct {
  int nc;
  double* b; /* 3*nc offsets of the control points from the centre (world frame) */
  double* k; /* nc positive weights */
  double c0[3];
  int motion; /* 0 static, 1 sinusoid, 2 constant velocity, 3 coupled (Eq. 4) */
  double amp[3], period, phase, vel[3];
  double rb;    /* bounding radius: M <= 1 beyond it */
  double cutsq; /* (rb + 2)^2: support of the solid fraction */
  /* two-way coupled particles (motion 3): offsets b are relative to the
   * centre of mass in the body frame; wb[0] holds them rotated to the
   * current orientation, wb[1] a copy that the fluid update reads while
   * the particle update rotates wb[0] */
  double* wb[2];
  double mass, Ib[3][3], Ibinv[3][3], cin; /* cin: level of the inner metaball */
  double c[3], v[3], q[4], L[3], w[3];     /* state at the domain's time */
  double Fh[3], Th[3];                      /* hydrodynamic force and torque of the last fluid update */
  int64_t acc[6];                           /* their fixed-point sums */
  int64_t acc_ibb[6];                       /* bounce-back coupling: sums of the last streaming */
} OPart;

typedef struct {
  int n[3];
  int bc[3];           /* 0 periodic, 1 wall pair */
  double wu[3][2][3];  /* velocity of the lo / hi wall of each wall axis */
  double tau, F[3], D, rho0, u0[3], sD;
  uint32_t key[2];
  int64_t N;
  double *f, *fs;                   /* [19][N] pre-collision, post-collision */
  double *rho, *u, *eps, *us;       /* rho[N], u[3][N], eps[N], us[3][N] */
  unsigned char* wall;              /* 1 on wall nodes */
  double* wallu;                    /* [3][N] wall velocity on wall nodes */
  OPart P[ORC_MAXP];
  int np;
  int64_t nw;
  int32_t *cell, *img; /* cell index; image counts [3][nw] */
  double* off;         /* [3][nw] offsets in [0,1) */
  double ref[3];
  int64_t t;
  uint64_t cnt[ORC_NCNT];
  int max_bisect;
  int seeded;
  /* two-way coupling of particles with motion 3 (Sec. 2.2, Eq. 4-11) */
  int ndem;
  double rho_p, g[3], drive_amp, drive_period, drive_dir[3], kn, kt, eta_n, eta_t, mu, Rs;
  int nsub, coupling;
  double xi[ORC_MAXP][ORC_MAXP][3]; /* tangential springs of particle pairs (i < j) */
  double xiw[ORC_MAXP][6][3];       /* and of particle-wall contacts */
  /* interpolated bounce-back coupling (Sec. 2.4.3, Eq. 23-27) instead of the
   * partially saturated cells: node status (0 fluid, p + 1 inside particle
   * p) at the poses of the current and of the previous fluid update */
  int ibb;
  int32_t *smap, *smap_prev;
} orc_domain;

static void dem_accumulate(orc_domain* d, const void* Pt, const int nd[3], const double* ep, double es,
                           const double fx[3]);

enum { C_TYPE2 = 0, C_TYPE4, C_BISECT_FAIL, C_REFILL_FALLBACK, C_RETURNED, C_WALL_REFLECT };

static int64_t nidx(const orc_domain* d, int x, int y, int z) {
  return (int64_t)x + (int64_t)d->n[0] * ((int64_t)y + (int64_t)d->n[1] * (int64_t)z);
}

orc_domain* orc_create(const int n[3], const int bc[3], const double wall_lo[9],
                       const double wall_hi[9], double tau, const double F[3], double D,
                       double rho0, const double u0[3], uint64_t seed) {
  init_weights();
  orc_domain* d = (orc_domain*)calloc(1, sizeof(orc_domain));
  for (int a = 0; a < 3; a++) {
    d->n[a] = n[a];
    d->bc[a] = bc[a];
    for (int c = 0; c < 3; c++) {
      d->wu[a][0][c] = wall_lo[3 * a + c];
      d->wu[a][1][c] = wall_hi[3 * a + c];
    }
    d->F[a] = F[a];
    d->u0[a] = u0[a];
  }
  d->tau = tau;
  d->D = D;
  d->sD = sqrt(2.0 * D);
  d->rho0 = rho0;
  d->key[0] = (uint32_t)seed;
  d->key[1] = (uint32_t)(seed >> 32);
  d->max_bisect = 200;
  d->N = (int64_t)n[0] * n[1] * n[2];
  int64_t N = d->N;
  d->f = (double*)malloc(sizeof(double) * 19 * N);
  d->fs = (double*)malloc(sizeof(double) * 19 * N);
  d->rho = (double*)malloc(sizeof(double) * N);
  d->u = (double*)malloc(sizeof(double) * 3 * N);
  d->eps = (double*)calloc(N, sizeof(double));
  d->us = (double*)calloc(3 * N, sizeof(double));
  d->wall = (unsigned char*)calloc(N, 1);
  d->wallu = (double*)calloc(3 * N, sizeof(double));
  for (int z = 0; z < n[2]; z++)
    for (int y = 0; y < n[1]; y++)
      for (int x = 0; x < n[0]; x++) {
        int64_t id = nidx(d, x, y, z);
        int co[3] = {x, y, z};
        for (int a = 0; a < 3 && !d->wall[id]; a++) {
          if (!bc[a]) continue;
          int side = co[a] == 0 ? 0 : (co[a] == n[a] - 1 ? 1 : -1);
          if (side < 0) continue;
          d->wall[id] = 1;
          for (int c = 0; c < 3; c++) d->wallu[c * N + id] = d->wu[a][side][c];
        }
        for (int i = 0; i < 19; i++) d->f[i * N + id] = feq(i, rho0, u0);
        d->rho[id] = rho0;
        for (int c = 0; c < 3; c++)
          d->u[c * N + id] = d->wall[id] ? d->wallu[c * N + id] : u0[c];
      }
  return d;
}

void orc_destroy(orc_domain* d) {
  if (!d) return;
  free(d->f); free(d->fs); free(d->rho); free(d->u); free(d->eps); free(d->us);
  free(d->wall); free(d->wallu);
  for (int p = 0; p < d->np; p++) { free(d->P[p].b); free(d->P[p].k); free(d->P[p].wb[0]); free(d->P[p].wb[1]); }
  free(d->cell); free(d->img); free(d->off);
  free(d->smap); free(d->smap_prev);
  free(d);
}

void orc_set_max_bisect(orc_domain* d, int m) { d->max_bisect = m; }

/* Bounding radius: with K = sum k_i and R_b = max |b_i| + sqrt(K), every
 * control point is at least sqrt(K) away from any x with |x - c| >= R_b, so
 * M(x) <= sum k_i / K = 1 there. */
int orc_add_particle(orc_domain* d, int nc, const double* b, const double* k,
                     const double c0[3], int motion, const double amp[3], double period,
                     double phase, const double vel[3]) {
  if (d->np >= ORC_MAXP || nc < 1) return -1;
  OPart* p = &d->P[d->np];
  p->nc = nc;
  p->b = (double*)malloc(sizeof(double) * 3 * nc);
  p->k = (double*)malloc(sizeof(double) * nc);
  memcpy(p->b, b, sizeof(double) * 3 * nc);
  memcpy(p->k, k, sizeof(double) * nc);
  double K = 0.0, bmax = 0.0;
  for (int i = 0; i < nc; i++) {
    K = K + k[i];
    double r = sqrt(b[3 * i] * b[3 * i] + b[3 * i + 1] * b[3 * i + 1] + b[3 * i + 2] * b[3 * i + 2]);
    if (r > bmax) bmax = r;
  }
  p->rb = bmax + sqrt(K);
  p->cutsq = (p->rb + 2.0) * (p->rb + 2.0);
  for (int a = 0; a < 3; a++) {
    p->c0[a] = c0[a];
    p->amp[a] = amp ? amp[a] : 0.0;
    p->vel[a] = vel ? vel[a] : 0.0;
  }
  p->motion = motion;
  p->period = period;
  p->phase = phase;
  return d->np++;
}

/* Prescribed rigid motion.  Sinusoid: c(t) = c0 + A sin(2 pi (t/T + phase)),
 * v(t) = A (2 pi / T) cos(...), phase in cycles; constant velocity:
 * c(t) = c0 + v t.  Orientation is fixed (no rotation), so the rigid surface
 * velocity v_p + w x (x - x_p) of Sec. 2.4.3 reduces to v_p. */
static void pose(const OPart* p, int64_t t, double c[3], double v[3]) {
  if (p->motion == 1) {
    double ph = (double)t / p->period + p->phase;
    ph = ph - floor(ph);
    double s, co;
    sincos2pi(ph, &s, &co);
    double w = 0x1.921fb54442d18p+2 / p->period; /* 2 pi / T */
    for (int a = 0; a < 3; a++) {
      c[a] = p->c0[a] + p->amp[a] * s;
      v[a] = (p->amp[a] * w) * co;
    }
  } else if (p->motion == 2) {
    for (int a = 0; a < 3; a++) {
      c[a] = p->c0[a] + p->vel[a] * (double)t;
      v[a] = p->vel[a];
    }
  } else {
    for (int a = 0; a < 3; a++) { c[a] = p->c0[a]; v[a] = 0.0; }
  }
}

/* Poses of every particle at one time: centre, velocity, angular velocity
 * and the control-point offsets in the world frame. */
typedef struct {
  double c[ORC_MAXP][3], v[ORC_MAXP][3], w[ORC_MAXP][3];
  const double* b[ORC_MAXP];
} Poses;

/* Prescribed particles: the pose at t; coupled particles (motion 3): the
 * current state (or the next one with `next`, once the step's particle
 * update has run). */
static void all_poses_which(const orc_domain* d, int64_t t, int next, Poses* P) {
  for (int p = 0; p < d->np; p++) {
    const OPart* q = &d->P[p];
    if (q->motion == 3) {
      for (int a = 0; a < 3; a++) {
        P->c[p][a] = q->c[a];
        P->v[p][a] = q->v[a];
        P->w[p][a] = q->w[a];
      }
      P->b[p] = q->wb[next];
    } else {
      pose(q, t, P->c[p], P->v[p]);
      for (int a = 0; a < 3; a++) P->w[p][a] = 0.0;
      P->b[p] = q->b;
    }
  }
}

static void all_poses(const orc_domain* d, int64_t t, Poses* P) { all_poses_which(d, t, 0, P); }

/* Displacement from a particle centre to the point (cell + x) along axis a,
 * minimum image on periodic axes. */
static double rel(const orc_domain* d, int a, int cell_a, double cp, double x) {
  double r = ((double)cell_a - cp) + x;
  if (!d->bc[a]) {
    double L = (double)d->n[a];
    r = r - L * floor(r / L + 0.5);
  }
  return r;
}

/* Eq. 3: M = sum_i k_i / |x - x_i|^2, in control-point order (b: the
 * control points' offsets from the centre in the world frame). */
static double mb_Mb(const double* b, const double* k, int nc, const double dl[3]) {
  double M = 0.0;
  for (int i = 0; i < nc; i++) {
    double rx = dl[0] - b[3 * i], ry = dl[1] - b[3 * i + 1], rz = dl[2] - b[3 * i + 2];
    double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == 0.0) return INFINITY;
    M = M + k[i] / r2;
  }
  return M;
}

/* Eq. 17: grad M = sum_i -2 k_i (x - x_i) / |x - x_i|^4. */
static void mb_gradb(const double* b, const double* k, int nc, const double dl[3], double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  for (int i = 0; i < nc; i++) {
    double r[3] = {dl[0] - b[3 * i], dl[1] - b[3 * i + 1], dl[2] - b[3 * i + 2]};
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double q = (-2.0 * k[i]) / (r2 * r2);
    for (int a = 0; a < 3; a++) g[a] = g[a] + q * r[a];
  }
}

static double mb_M(const OPart* p, const double dl[3]) { return mb_Mb(p->b, p->k, p->nc, dl); }
static void mb_grad(const OPart* p, const double dl[3], double g[3]) { mb_gradb(p->b, p->k, p->nc, dl, g); }

static void delta_to(const orc_domain* d, const Poses* P, int p, const int cell[3],
                     const double x[3], double dl[3]) {
  for (int a = 0; a < 3; a++) dl[a] = rel(d, a, cell[a], P->c[p][a], x[a]);
}

static double M_at(const orc_domain* d, const Poses* P, int p, const int cell[3], const double x[3]) {
  double dl[3];
  delta_to(d, P, p, cell, x, dl);
  return mb_Mb(P->b[p], d->P[p].k, d->P[p].nc, dl);
}

static void grad_at(const orc_domain* d, const Poses* P, int p, const double dl[3], double g[3]) {
  mb_gradb(P->b[p], d->P[p].k, d->P[p].nc, dl, g);
}

/* Inside a particle <=> its own M >= 1 (each particle has its own function);
 * returns the lowest such particle index, or -1. */
static int inside_any(const orc_domain* d, const Poses* P, const int cell[3], const double x[3]) {
  for (int p = 0; p < d->np; p++)
    if (M_at(d, P, p, cell, x) >= 1.0) return p;
  return -1;
}

/* Solid fraction of one particle at a node: 1/2 + d clamped to [0,1], with d
 * the signed distance (positive inside) to the surface estimated from the
 * field M^(-1/2), whose level 1 is the surface:
 *   d = (1 - M^(-1/2)) / |grad M^(-1/2)| = 2 M (sqrt(M) - 1) / |grad M|.
 * Near the surface this is the first-order estimate (M - 1)/|grad M|; for a
 * single control point it is the exact distance sqrt(k) - r.  Zero outside
 * the support |x - c| > R_b + 2. */
static double eps_one(const orc_domain* d, const Poses* P, int p, const int nd[3]) {
  const OPart* q = &d->P[p];
  double dl[3];
  for (int a = 0; a < 3; a++) dl[a] = rel(d, a, nd[a], P->c[p][a], 0.5);
  double r2c = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
  if (r2c > q->cutsq) return 0.0;
  double M = mb_Mb(P->b[p], q->k, q->nc, dl);
  if (M == INFINITY) return 1.0;
  double g[3];
  mb_gradb(P->b[p], q->k, q->nc, dl, g);
  double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  double e;
  if (gn == 0.0) {
    e = M >= 1.0 ? 1.0 : 0.0;
  } else {
    double dist = ((2.0 * M) * (sqrt(M) - 1.0)) / gn;
    e = dist == dist ? 0.5 + dist : (M >= 1.0 ? 1.0 : 0.0);
  }
  if (e < 0.0) e = 0.0;
  if (e > 1.0) e = 1.0;
  return e;
}

/* ------------------------------------------------------------ fluid */
/* Collision at one node (pre-collision f[19] in, post-collision out[19]).
 * rho = sum f_i, j = sum f_i e_i (Eq. 14-15), u = (j + F/2)/rho (Guo).
 * B = eps (tau - 1/2) / ((1 - eps) + (tau - 1/2));
 * Om_i = [f_opp - feq_opp(rho,u)] - [f_i - feq_i(rho,us)];
 * S_i = w_i [3 (e_i - u).F + 9 (e_i.u)(e_i.F)];
 * f*_i = f_i - (1-B)/tau (f_i - feq_i(rho,u)) + B Om_i + (1-B)(1 - 1/(2 tau)) S_i. */
static void collide_node_x(const orc_domain* d, const double f[19], double eps, const double us[3],
                           double out[19], double* rho_out, double u_out[3], double fx[3]);
static void collide_node(const orc_domain* d, const double f[19], double eps, const double us[3],
                         double out[19], double* rho_out, double u_out[3]) {
  double fx[3];
  collide_node_x(d, f, eps, us, out, rho_out, u_out, fx);
}

/* The same collision, also returning the momentum the solid term takes from
 * the fluid: fx = -sum_i B Om_i e_i (index order), the node's share of the
 * hydrodynamic force on the particles (momentum exchange of the partially
 * saturated cells). */
static void collide_node_x(const orc_domain* d, const double f[19], double eps, const double us[3],
                           double out[19], double* rho_out, double u_out[3], double fx[3]) {
  double rho = 0.0;
  for (int i = 0; i < 19; i++) rho = rho + f[i];
  double j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 19; i++)
    for (int a = 0; a < 3; a++) {
      if (EV[i][a] == 1) j[a] = j[a] + f[i];
      else if (EV[i][a] == -1) j[a] = j[a] - f[i];
    }
  double u[3];
  for (int a = 0; a < 3; a++) u[a] = (j[a] + 0.5 * d->F[a]) / rho;
  double omega = 1.0 / d->tau;
  double tm = d->tau - 0.5;
  double B = (eps * tm) / ((1.0 - eps) + tm);
  double A = (1.0 - B) * omega;
  double Cf = (1.0 - B) * (1.0 - 0.5 * omega);
  double fe[19], fes[19];
  for (int i = 0; i < 19; i++) {
    fe[i] = feq(i, rho, u);
    fes[i] = feq(i, rho, us);
  }
  double fxa[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 19; i++) {
    int o = opp(i);
    double Om = (f[o] - fe[o]) - (f[i] - fes[i]);
    double eu = edot(i, u);
    double eF = edot(i, d->F);
    double emF = 0.0;
    for (int a = 0; a < 3; a++) emF = emF + ((double)EV[i][a] - u[a]) * d->F[a];
    double S = WT[i] * (3.0 * emF + (9.0 * eu) * eF);
    double bo = B * Om;
    out[i] = ((f[i] - A * (f[i] - fe[i])) + bo) + Cf * S;
    for (int a = 0; a < 3; a++) {
      if (EV[i][a] == 1) fxa[a] = fxa[a] - bo;
      else if (EV[i][a] == -1) fxa[a] = fxa[a] + bo;
    }
  }
  for (int a = 0; a < 3; a++) fx[a] = fxa[a];
  *rho_out = rho;
  for (int a = 0; a < 3; a++) u_out[a] = u[a];
}

static void fluid_step_ibb(orc_domain* d, const Poses* Pt);

static void fluid_step(orc_domain* d, const Poses* Pt) {
  if (d->ibb) {
    fluid_step_ibb(d, Pt);
    return;
  }
  const int64_t N = d->N;
  const int nx = d->n[0], ny = d->n[1], nz = d->n[2];
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < N; id++) {
    if (d->wall[id]) continue;
    int nd[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((int64_t)nx * ny))};
    /* solid fraction and solid velocity: eps = min(1, sum eps_p),
     * us = sum eps_p v_p / sum eps_p (particle order) */
    double es = 0.0, un[3] = {0.0, 0.0, 0.0}, ep[ORC_MAXP];
    for (int p = 0; p < d->np; p++) {
      double e = eps_one(d, Pt, p, nd);
      ep[p] = e;
      es = es + e;
      double up[3] = {Pt->v[p][0], Pt->v[p][1], Pt->v[p][2]};
      if (d->P[p].motion == 3 && e > 0.0) {
        /* rigid surface velocity v + w x (x - x_p) (Sec. 2.4.3) */
        double dl[3];
        for (int a = 0; a < 3; a++) dl[a] = rel(d, a, nd[a], Pt->c[p][a], 0.5);
        const double* w = Pt->w[p];
        up[0] = up[0] + (w[1] * dl[2] - w[2] * dl[1]);
        up[1] = up[1] + (w[2] * dl[0] - w[0] * dl[2]);
        up[2] = up[2] + (w[0] * dl[1] - w[1] * dl[0]);
      }
      for (int a = 0; a < 3; a++) un[a] = un[a] + e * up[a];
    }
    double eps = es < 1.0 ? es : 1.0;
    double us[3];
    for (int a = 0; a < 3; a++) us[a] = es > 0.0 ? un[a] / es : 0.0;
    double f[19], out[19], rho, u[3], fx[3];
    for (int i = 0; i < 19; i++) f[i] = d->f[i * N + id];
    collide_node_x(d, f, eps, us, out, &rho, u, fx);
    if (d->ndem > 0 && es > 0.0) dem_accumulate(d, Pt, nd, ep, es, fx);
    for (int i = 0; i < 19; i++) d->fs[i * N + id] = out[i];
    d->rho[id] = rho;
    d->eps[id] = eps;
    for (int a = 0; a < 3; a++) {
      d->u[a * N + id] = u[a];
      d->us[a * N + id] = us[a];
    }
  }
  /* streaming: f_i(x, t+1) = f*_i(x - e_i); from a wall node the population
   * is the bounced one, f*_opp(i)(x) + 6 w_i rho(x) (e_i . u_w) (Eq. 23 form) */
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < N; id++) {
    if (d->wall[id]) continue;
    int nd[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((int64_t)nx * ny))};
    for (int i = 0; i < 19; i++) {
      int s[3];
      for (int a = 0; a < 3; a++) {
        s[a] = nd[a] - EV[i][a];
        if (s[a] < 0) s[a] += d->n[a];
        if (s[a] >= d->n[a]) s[a] -= d->n[a];
      }
      int64_t sid = nidx(d, s[0], s[1], s[2]);
      (void)nz;
      if (d->wall[sid]) {
        double uw[3] = {d->wallu[sid], d->wallu[N + sid], d->wallu[2 * N + sid]};
        double term = ((6.0 * WT[i]) * d->rho[id]) * edot(i, uw);
        d->f[i * N + id] = d->fs[opp(i) * N + id] + term;
      } else {
        d->f[i * N + id] = d->fs[i * N + sid];
      }
    }
  }
}

/* ------------------------------------------------ interpolated bounce-back */
/* The paper's own fluid-particle rule (Sec. 2.4.3, Eq. 23-27), read for a
 * pull-free collide-then-stream update:
 *  - a node is solid when its centre is inside a particle (M_p >= 1, the
 *    lowest index wins), else fluid; solid nodes do not collide, their
 *    velocity is the particle's rigid velocity v + w x r and their density
 *    rho0 (for the walkers and the averages);
 *  - a node that was solid at the previous update and is fluid now is
 *    refilled with f^eq(rho0, u_new), u_new the rigid velocity of the
 *    particle that covered it (Eq. 27; the bounce-back refill of Eq. 26
 *    needs populations a formerly solid node does not have);
 *  - streaming after the collision at P(t): a fluid node x_f whose upstream
 *    node x_f - e_i is solid receives Eq. 23, G_i = G+_{i'}(x_d) + 6 w rho_f
 *    e_i . u_w, with Eq. 24 G+_{i'}(x_d) = f^eq_{i'}(rho_f, u_d) + the
 *    non-equilibrium part of x_f's own post-collision population i', Eq. 25
 *    for u_d, q the fraction of the link from x_f to the surface M = 1 (a
 *    bracketed regula falsi, ibb_q), u_w the rigid velocity at the surface point, u_ff
 *    the velocity at x_f + e_i (u_f where that node is a wall or solid);
 *  - the momentum exchange of each such link in its Galilean-invariant form,
 *    (e_i' - u_w) G+_i'(x_f) - (e_i - u_w) G_i, with its torque about the
 *    particle's centre, goes to a coupled particle; the particle update of
 *    the next step uses it. */

/* Lowest index of a particle whose M >= 1 at the centre of node nd, or -1. */
static int solid_at(const orc_domain* d, const Poses* P, const int nd[3]) {
  for (int p = 0; p < d->np; p++) {
    const OPart* q = &d->P[p];
    double dl[3];
    for (int a = 0; a < 3; a++) dl[a] = rel(d, a, nd[a], P->c[p][a], 0.5);
    double r2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
    if (!(r2 < q->rb * q->rb)) continue;
    if (mb_Mb(P->b[p], q->k, q->nc, dl) >= 1.0) return p;
  }
  return -1;
}

/* v + w x dl, the velocity of particle p's rigid body at offset dl. */
static void rigid_vel(const Poses* P, int p, const double dl[3], double up[3]) {
  const double* v = P->v[p];
  const double* w = P->w[p];
  up[0] = v[0] + (w[1] * dl[2] - w[2] * dl[1]);
  up[1] = v[1] + (w[2] * dl[0] - w[0] * dl[2]);
  up[2] = v[2] + (w[0] * dl[1] - w[1] * dl[0]);
}

/* Eq. 25: u_d from the velocities at x_f, x_ff and the wall point. */
static void ibb_ud(double q, const double uf[3], const double uff[3], const double uw[3], double ud[3]) {
  for (int a = 0; a < 3; a++) {
    double u1 = q <= 0.5 ? (2.0 * q) * uf[a] + (1.0 - 2.0 * q) * uff[a]
                         : ((1.0 - q) / q) * uf[a] + ((2.0 * q - 1.0) / q) * uw[a];
    double u2 = ((1.0 - q) / (1.0 + q)) * uff[a] + ((2.0 * q) / (1.0 + q)) * uw[a];
    ud[a] = u1 / 3.0 + (2.0 * u2) / 3.0;
  }
}

/* 1 - M^(-1/2) at fraction s of the link from offset d0 along e_o: the
 * distance-like field whose zero is the surface M = 1 (nearly linear along
 * a link, exactly so for a sphere seen radially). */
static double ibb_phi(const orc_domain* d, const Poses* P, int p, const double d0[3], int o, double s) {
  const OPart* q = &d->P[p];
  double x[3];
  for (int a = 0; a < 3; a++) x[a] = d0[a] + s * (double)EV[o][a];
  return 1.0 - 1.0 / sqrt(mb_Mb(P->b[p], q->k, q->nc, x));
}

/* q of the link from the centre of node nd along e_o into particle p: the
 * root of 1 - M^(-1/2) between q = 0 (M < 1, a fluid node) and q = 1
 * (M >= 1, a node inside p), by the Illinois variant of regula falsi, ten
 * steps or until the field is exactly zero (the bracket always holds a
 * sign change); dlw receives the surface point's offset from p's centre. */
static double ibb_q(const orc_domain* d, const Poses* P, int p, const int nd[3], int o, double dlw[3]) {
  double d0[3];
  for (int a = 0; a < 3; a++) d0[a] = rel(d, a, nd[a], P->c[p][a], 0.5);
  double a0 = 0.0, b0 = 1.0;
  double fa = ibb_phi(d, P, p, d0, o, a0), fb = ibb_phi(d, P, p, d0, o, b0);
  for (int it = 0; it < 10; it++) {
    if (fb == fa) break;
    double c = b0 - fb * ((b0 - a0) / (fb - fa));
    double fc = ibb_phi(d, P, p, d0, o, c);
    if (fc == 0.0) {
      b0 = c;
      break;
    }
    if ((fc < 0.0) == (fb < 0.0)) fa = 0.5 * fa;
    else {
      a0 = b0;
      fa = fb;
    }
    b0 = c;
    fb = fc;
  }
  double qq = b0;
  for (int a = 0; a < 3; a++) dlw[a] = d0[a] + qq * (double)EV[o][a];
  return qq;
}

static int64_t fix48(double x);

static void fluid_step_ibb(orc_domain* d, const Poses* Pt) {
  const int64_t N = d->N;
  const int nx = d->n[0], ny = d->n[1];
  int32_t* tmp = d->smap_prev;
  d->smap_prev = d->smap;
  d->smap = tmp;
  int32_t* sm = d->smap;
  const int32_t* sp = d->smap_prev;
  /* collision at P(t) */
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < N; id++) {
    if (d->wall[id]) {
      sm[id] = 0;
      continue;
    }
    int nd[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((int64_t)nx * ny))};
    int s = solid_at(d, Pt, nd);
    sm[id] = s + 1;
    if (s >= 0) {
      double dl[3], up[3];
      for (int a = 0; a < 3; a++) dl[a] = rel(d, a, nd[a], Pt->c[s][a], 0.5);
      rigid_vel(Pt, s, dl, up);
      d->rho[id] = d->rho0;
      d->eps[id] = 1.0;
      for (int a = 0; a < 3; a++) {
        d->u[a * N + id] = up[a];
        d->us[a * N + id] = up[a];
      }
      continue;
    }
    double f[19], out[19], rho, u[3];
    const double zero[3] = {0.0, 0.0, 0.0};
    if (sp[id] > 0) { /* uncovered since the last update: Eq. 27 */
      int pp = sp[id] - 1;
      double dl[3], un[3];
      for (int a = 0; a < 3; a++) dl[a] = rel(d, a, nd[a], Pt->c[pp][a], 0.5);
      rigid_vel(Pt, pp, dl, un);
      for (int i = 0; i < 19; i++) f[i] = feq(i, d->rho0, un);
    } else {
      for (int i = 0; i < 19; i++) f[i] = d->f[i * N + id];
    }
    collide_node(d, f, 0.0, zero, out, &rho, u);
    for (int i = 0; i < 19; i++) d->fs[i * N + id] = out[i];
    d->rho[id] = rho;
    d->eps[id] = 0.0;
    for (int a = 0; a < 3; a++) {
      d->u[a * N + id] = u[a];
      d->us[a * N + id] = 0.0;
    }
  }
  /* streaming with the boundary at P(t) */
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < N; id++) {
    if (d->wall[id] || sm[id] > 0) continue;
    int nd[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((int64_t)nx * ny))};
    const double rf = d->rho[id];
    const double uf[3] = {d->u[id], d->u[N + id], d->u[2 * N + id]};
    for (int i = 0; i < 19; i++) {
      int s3[3], f3[3];
      for (int a = 0; a < 3; a++) {
        s3[a] = nd[a] - EV[i][a];
        if (s3[a] < 0) s3[a] += d->n[a];
        if (s3[a] >= d->n[a]) s3[a] -= d->n[a];
        f3[a] = nd[a] + EV[i][a];
        if (f3[a] < 0) f3[a] += d->n[a];
        if (f3[a] >= d->n[a]) f3[a] -= d->n[a];
      }
      int64_t sid = nidx(d, s3[0], s3[1], s3[2]);
      const int o = opp(i);
      if (d->wall[sid]) {
        double uw[3] = {d->wallu[sid], d->wallu[N + sid], d->wallu[2 * N + sid]};
        double term = ((6.0 * WT[i]) * rf) * edot(i, uw);
        d->f[i * N + id] = d->fs[o * N + id] + term;
      } else if (sm[sid] > 0) {
        int p = sm[sid] - 1;
        double dlw[3], uw[3], uff[3], ud[3];
        double q = ibb_q(d, Pt, p, nd, o, dlw);
        rigid_vel(Pt, p, dlw, uw);
        int64_t fid = nidx(d, f3[0], f3[1], f3[2]);
        for (int a = 0; a < 3; a++) uff[a] = (d->wall[fid] || sm[fid] > 0) ? uf[a] : d->u[a * N + fid];
        ibb_ud(q, uf, uff, uw, ud);
        double fso = d->fs[o * N + id];
        double gneq = fso - feq(o, rf, uf);
        double fi = (feq(o, rf, ud) + gneq) + ((6.0 * WT[o]) * rf) * edot(i, uw);
        d->f[i * N + id] = fi;
        if (d->P[p].motion == 3) {
          double F[3];
          for (int a = 0; a < 3; a++)
            F[a] = ((double)EV[o][a] - uw[a]) * fso - ((double)EV[i][a] - uw[a]) * fi;
          double T[3] = {dlw[1] * F[2] - dlw[2] * F[1], dlw[2] * F[0] - dlw[0] * F[2], dlw[0] * F[1] - dlw[1] * F[0]};
          int64_t v[6] = {fix48(F[0]), fix48(F[1]), fix48(F[2]), fix48(T[0]), fix48(T[1]), fix48(T[2])};
          for (int k = 0; k < 6; k++) {
#pragma omp atomic
            d->P[p].acc_ibb[k] += v[k];
          }
        }
      } else {
        d->f[i * N + id] = d->fs[i * N + sid];
      }
    }
  }
}

/* Interpolated bounce-back instead of partially saturated cells; before the
 * first step. */
int orc_set_ibb(orc_domain* d, int on) {
  if (d->t != 0) return -1;
  d->ibb = on ? 1 : 0;
  if (d->ibb && !d->smap) {
    d->smap = (int32_t*)calloc(d->N, sizeof(int32_t));
    d->smap_prev = (int32_t*)calloc(d->N, sizeof(int32_t));
  }
  return 0;
}

/* Eq. 25 alone (for tests). */
void orc_ibb_ud(double q, const double uf[3], const double uff[3], const double uw[3], double ud[3]) {
  ibb_ud(q, uf, uff, uw, ud);
}

/* q and the surface point of the link from node cell along e_o into particle
 * p at step t (for tests). */
double orc_ibb_q(const orc_domain* d, int p, int64_t t, const int cell[3], int o, double dlw[3]) {
  Poses P;
  all_poses(d, t, &P);
  return ibb_q(d, &P, p, cell, o, dlw);
}

/* Node status of the last fluid update: 0 fluid, p + 1 inside particle p. */
void orc_get_smap(const orc_domain* d, int32_t* out) {
  if (d->smap) memcpy(out, d->smap, sizeof(int32_t) * d->N);
  else memset(out, 0, sizeof(int32_t) * d->N);
}

/* ----------------------------------------------------------- walkers */
/* Algorithm 1 on the straight segment x(s) = a + s dir, s from s_out (M<1)
 * to s_in (M>=1): midpoint in s, stop when |M - 1| < 1e-3, at most imax
 * evaluations.  Returns 1 and the converged s on success. */
static int bisect(const orc_domain* d, const Poses* P, int p, const int cell[3], const double a0[3],
                  const double dir[3], double s_out, double s_in, int imax, double* s_res) {
  for (int it = 1; it <= imax; it++) {
    double sm = 0.5 * (s_out + s_in);
    double x[3];
    for (int a = 0; a < 3; a++) x[a] = a0[a] + sm * dir[a];
    double m = M_at(d, P, p, cell, x);
    if (fabs(m - 1.0) < 1e-3) {
      *s_res = sm;
      return 1;
    }
    if (m < 1.0) s_out = sm;
    else s_in = sm;
  }
  return 0;
}

static double prev_double(double x) { /* x > 0 */
  uint64_t b;
  memcpy(&b, &x, 8);
  b -= 1;
  memcpy(&x, &b, 8);
  return x;
}

typedef struct { uint64_t c[ORC_NCNT]; } Cnt;

/* One walker, one step.  cell/x are the walker's cell and offset (updated in
 * place, with image counts), u(t) is the fluid velocity of this step, Pn the
 * particle poses at t+1. */
static void walker_step(const orc_domain* d, const Poses* Pn, int64_t w, int cell[3], double o[3],
                        int img[3], Cnt* cn) {
  const int64_t N = d->N;
  const int* n = d->n;
  /* 1. trilinear interpolation between node centres, x then y then z */
  int b0[3], b1[3];
  double wt[3];
  for (int a = 0; a < 3; a++) {
    int b;
    if (o[a] >= 0.5) { b = cell[a]; wt[a] = o[a] - 0.5; }
    else { b = cell[a] - 1; wt[a] = o[a] + 0.5; }
    int c1 = b + 1;
    if (b < 0) b += n[a];
    if (c1 >= n[a]) c1 -= n[a];
    b0[a] = b;
    b1[a] = c1;
  }
  double U[3];
  for (int c = 0; c < 3; c++) {
    const double* uc = d->u + c * N;
    double v[2][2];
    for (int zz = 0; zz < 2; zz++)
      for (int yy = 0; yy < 2; yy++) {
        int y = yy ? b1[1] : b0[1], z = zz ? b1[2] : b0[2];
        double lo = uc[nidx(d, b0[0], y, z)], hi = uc[nidx(d, b1[0], y, z)];
        v[zz][yy] = (1.0 - wt[0]) * lo + wt[0] * hi;
      }
    double v0 = (1.0 - wt[1]) * v[0][0] + wt[1] * v[0][1];
    double v1 = (1.0 - wt[1]) * v[1][0] + wt[1] * v[1][1];
    U[c] = (1.0 - wt[2]) * v0 + wt[2] * v1;
  }
  /* 2-3. Eq. 2 with dt = 1: x_f = x_p + u + z sqrt(2D) */
  uint32_t ctr[4] = {(uint32_t)w, (uint32_t)d->t, 0u, 0u}, r[4];
  philox(ctr, d->key, r);
  double z[3], dl[3], xf[3];
  normals3(r, z);
  for (int a = 0; a < 3; a++) {
    dl[a] = U[a] + z[a] * d->sD;
    xf[a] = o[a] + dl[a];
  }
  /* 4. walker/particle relation at the next pose (types I-IV) */
  double xn[3];
  for (int a = 0; a < 3; a++) xn[a] = xf[a];
  int jb = inside_any(d, Pn, cell, xf);
  if (jb >= 0) {
    int ja = inside_any(d, Pn, cell, o);
    if (ja < 0) {
      /* type IV: no-flux, Algorithm 1 then Algorithm 2 */
      cn->c[C_TYPE4]++;
      double s;
      int ok = bisect(d, Pn, jb, cell, o, dl, 0.0, 1.0, d->max_bisect, &s);
      int done = 0;
      if (ok) {
        double xi[3], dv[3], g[3];
        for (int a = 0; a < 3; a++) xi[a] = o[a] + s * dl[a];
        delta_to(d, Pn, jb, cell, xi, dv);
        grad_at(d, Pn, jb, dv, g);
        double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        if (gn > 0.0) {
          double nv[3], ti[3];
          for (int a = 0; a < 3; a++) {
            nv[a] = g[a] / gn;
            ti[a] = xf[a] - xi[a];
          }
          double dt = ti[0] * nv[0] + ti[1] * nv[1] + ti[2] * nv[2];
          for (int a = 0; a < 3; a++) xn[a] = xi[a] + (ti[a] - (2.0 * dt) * nv[a]);
          if (inside_any(d, Pn, cell, xn) >= 0) {
            cn->c[C_RETURNED]++;
            for (int a = 0; a < 3; a++) xn[a] = o[a];
          }
          done = 1;
        }
      }
      if (!done) {
        cn->c[C_BISECT_FAIL]++;
        for (int a = 0; a < 3; a++) xn[a] = o[a];
      }
    } else {
      /* type II: refill -- push out along -grad M, place at random within
       * the sqrt(2D) half-ball outside the surface */
      cn->c[C_TYPE2]++;
      double dv[3], g[3];
      delta_to(d, Pn, jb, cell, xf, dv);
      grad_at(d, Pn, jb, dv, g);
      double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
      int fallback = 1;
      if (gn > 0.0) {
        double no[3];
        for (int a = 0; a < 3; a++) no[a] = (-g[a]) / gn;
        double s = 0.5, lim = 2.0 * d->P[jb].rb;
        double xe[3];
        for (;;) {
          for (int a = 0; a < 3; a++) xe[a] = xf[a] + s * no[a];
          if (!(M_at(d, Pn, jb, cell, xe) >= 1.0) || !(s < lim)) break;
          s = 2.0 * s;
        }
        if (M_at(d, Pn, jb, cell, xe) < 1.0) {
          double ss;
          int ok = bisect(d, Pn, jb, cell, xf, no, s, 0.0, d->max_bisect, &ss);
          double xs[3];
          if (ok) {
            for (int a = 0; a < 3; a++) xs[a] = xf[a] + ss * no[a];
            uint32_t c1[4] = {(uint32_t)w, (uint32_t)d->t, 1u, 0u}, r1[4];
            uint32_t c2[4] = {(uint32_t)w, (uint32_t)d->t, 2u, 0u}, r2[4];
            philox(c1, d->key, r1);
            philox(c2, d->key, r2);
            double v[3];
            normals3(r1, v);
            double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            for (int a = 0; a < 3; a++) v[a] = v[a] / vn;
            if (v[0] * no[0] + v[1] * no[1] + v[2] * no[2] < 0.0)
              for (int a = 0; a < 3; a++) v[a] = -v[a];
            double mx = u01(r2[0]);
            if (u01(r2[1]) > mx) mx = u01(r2[1]);
            if (u01(r2[2]) > mx) mx = u01(r2[2]);
            double rr = d->sD * mx;
            for (int a = 0; a < 3; a++) xn[a] = xs[a] + rr * v[a];
          } else {
            cn->c[C_BISECT_FAIL]++;
            for (int a = 0; a < 3; a++) xn[a] = xe[a];
          }
          int bad = inside_any(d, Pn, cell, xn) >= 0;
          for (int a = 0; a < 3 && !bad; a++) {
            if (!d->bc[a]) continue;
            double lo = 1.0 - (double)cell[a], hi = (double)(n[a] - 1) - (double)cell[a];
            if (xn[a] < lo || xn[a] >= hi) bad = 1;
          }
          if (bad)
            for (int a = 0; a < 3; a++) xn[a] = xe[a];
          fallback = inside_any(d, Pn, cell, xn) >= 0;
        }
      }
      if (fallback) {
        cn->c[C_REFILL_FALLBACK]++;
        for (int a = 0; a < 3; a++) xn[a] = xf[a];
      }
    }
  }
  /* a non-finite position (only from an unstable flow) keeps the walker
   * where it was */
  if (!(isfinite(xn[0]) && isfinite(xn[1]) && isfinite(xn[2]))) {
    cn->c[C_RETURNED]++;
    for (int a = 0; a < 3; a++) xn[a] = o[a];
  }
  /* 5. walls: halfway planes at 1 and n-1 on wall axes, one specular
   * reflection per axis; a reflected point still outside the fluid range, or
   * inside a particle, returns the walker to where it started (narrow gaps) */
  int refl = 0;
  for (int a = 0; a < 3; a++) {
    if (!d->bc[a]) continue;
    double lo = 1.0 - (double)cell[a], hi = (double)(n[a] - 1) - (double)cell[a];
    if (xn[a] < lo) {
      xn[a] = 2.0 * lo - xn[a];
      refl = 1;
    } else if (xn[a] >= hi) {
      xn[a] = 2.0 * hi - xn[a];
      if (xn[a] == hi) xn[a] = prev_double(hi);
      refl = 1;
    }
  }
  if (refl) {
    cn->c[C_WALL_REFLECT]++;
    int out = 0;
    for (int a = 0; a < 3; a++) {
      if (!d->bc[a]) continue;
      double lo = 1.0 - (double)cell[a], hi = (double)(n[a] - 1) - (double)cell[a];
      if (xn[a] < lo || xn[a] >= hi) out = 1;
    }
    if (out || inside_any(d, Pn, cell, xn) >= 0) {
      cn->c[C_RETURNED]++;
      for (int a = 0; a < 3; a++) xn[a] = o[a];
    }
  }
  /* 6. back to (cell, offset in [0,1)), periodic wrap with image counts */
  for (int a = 0; a < 3; a++) {
    double k = floor(xn[a]);
    double of = xn[a] - k;
    if (of == 1.0) {
      of = 0.0;
      k = k + 1.0;
    }
    int c = cell[a] + (int)k;
    if (!d->bc[a]) {
      int q = c >= 0 ? c / n[a] : -((-c + n[a] - 1) / n[a]); /* floor(c / n) */
      c -= q * n[a];
      img[a] += q;
    }
    cell[a] = c;
    o[a] = of;
  }
}

static void walkers_step(orc_domain* d, const Poses* Pn) {
  const int64_t nw = d->nw;
  const int nx = d->n[0], ny = d->n[1];
  uint64_t tot[ORC_NCNT] = {0};
#pragma omp parallel
  {
    Cnt cn;
    memset(&cn, 0, sizeof(cn));
#pragma omp for schedule(static)
    for (int64_t w = 0; w < nw; w++) {
      int32_t lc = d->cell[w];
      int cell[3] = {lc % nx, (lc / nx) % ny, lc / (nx * ny)};
      double o[3] = {d->off[w], d->off[nw + w], d->off[2 * nw + w]};
      int img[3] = {d->img[w], d->img[nw + w], d->img[2 * nw + w]};
      walker_step(d, Pn, w, cell, o, img, &cn);
      d->cell[w] = (int32_t)nidx(d, cell[0], cell[1], cell[2]);
      for (int a = 0; a < 3; a++) {
        d->off[a * nw + w] = o[a];
        d->img[a * nw + w] = img[a];
      }
    }
#pragma omp critical
    for (int c = 0; c < ORC_NCNT; c++) tot[c] += cn.c[c];
  }
  for (int c = 0; c < ORC_NCNT; c++) d->cnt[c] += tot[c];
}

/* ------------------------------------------------- two-way coupling */
/* Particles with motion 3 move by the Newton-Euler equations (Eq. 4) under
 * gravity, the oscillator's drive (Eq. 37 as a horizontal acceleration
 * a cos(2 pi t / T)), the hydrodynamic force and torque of the fluid update
 * (the momentum the solid term of the partially saturated cells takes from
 * the fluid, summed over the particle's nodes) and contacts: sphero-metaball
 * particles (an inner metaball M >= cin dilated by a sphere of radius Rs),
 * their closest points by Newton-Raphson (Eq. 6-9, Eq. 10-11 for walls), a
 * linear spring-dashpot normal force and a tangential spring capped by
 * Coulomb friction (Eq. 5).  nsub substeps per fluid step, symplectic Euler
 * for positions and angular momentum, the orientation a unit quaternion. */

#define ORC_FIX 281474976710656.0 /* 2^48: fixed-point scale of the force sums */

static void quat_R(const double q[4], double R[3][3]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1.0 - 2.0 * (y * y + z * z); R[0][1] = 2.0 * (x * y - w * z);       R[0][2] = 2.0 * (x * z + w * y);
  R[1][0] = 2.0 * (x * y + w * z);       R[1][1] = 1.0 - 2.0 * (x * x + z * z); R[1][2] = 2.0 * (y * z - w * x);
  R[2][0] = 2.0 * (x * z - w * y);       R[2][1] = 2.0 * (y * z + w * x);       R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

static void rotate_offsets(const OPart* p, const double q[4], double* out) {
  double R[3][3];
  quat_R(q, R);
  for (int i = 0; i < p->nc; i++)
    for (int a = 0; a < 3; a++)
      out[3 * i + a] = (R[a][0] * p->b[3 * i] + R[a][1] * p->b[3 * i + 1]) + R[a][2] * p->b[3 * i + 2];
}

static int inv3(const double A[3][3], double X[3][3]) {
  double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  double det = (A[0][0] * c00 + A[0][1] * c01) + A[0][2] * c02;
  if (det == 0.0 || !isfinite(det)) return -1;
  X[0][0] = c00 / det;
  X[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
  X[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
  X[1][0] = c01 / det;
  X[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
  X[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
  X[2][0] = c02 / det;
  X[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
  X[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
  return 0;
}

/* Solid fraction of a cell of size h centred at offset x (the first-order
 * distance estimate of the solid fraction, on the cell's scale). */
static double cell_fraction(const OPart* p, const double x[3], double h) {
  double M = mb_M(p, x);
  if (M == INFINITY) return 1.0;
  double g[3];
  mb_grad(p, x, g);
  double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  double e;
  if (gn == 0.0) e = M >= 1.0 ? 1.0 : 0.0;
  else e = 0.5 + (((2.0 * M) * (sqrt(M) - 1.0)) / gn) / h;
  if (!(e > 0.0)) e = 0.0;
  if (e > 1.0) e = 1.0;
  return e;
}

/* Mass, centre of mass and inertia tensor of a metaball of density rho_p:
 * cells of size h = rb/24 over the cube [-rb - h, rb + h]^3 about the reference
 * point (one cell beyond rb), each weighted by its solid fraction, summed
 * z, y, x in order. */
static void mass_properties(const OPart* p, double rho_p, double* mass, double com[3], double I[3][3]) {
  const int G = 50; /* cells of the cube [-rb - h, rb + h]^3 */
  const double h = p->rb / 24.0;
  double V = 0.0, S[3] = {0, 0, 0};
  for (int iz = 0; iz < G; iz++)
    for (int iy = 0; iy < G; iy++)
      for (int ix = 0; ix < G; ix++) {
        double x[3] = {((double)(ix - 25) + 0.5) * h, ((double)(iy - 25) + 0.5) * h, ((double)(iz - 25) + 0.5) * h};
        double e = cell_fraction(p, x, h);
        V = V + e;
        for (int a = 0; a < 3; a++) S[a] = S[a] + e * x[a];
      }
  for (int a = 0; a < 3; a++) com[a] = S[a] / V;
  double Q[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int iz = 0; iz < G; iz++)
    for (int iy = 0; iy < G; iy++)
      for (int ix = 0; ix < G; ix++) {
        double x[3] = {((double)(ix - 25) + 0.5) * h, ((double)(iy - 25) + 0.5) * h, ((double)(iz - 25) + 0.5) * h};
        double e = cell_fraction(p, x, h);
        double r[3] = {x[0] - com[0], x[1] - com[1], x[2] - com[2]};
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) Q[a][b] = Q[a][b] + e * (r[a] * r[b]);
      }
  double h3 = (h * h) * h;
  *mass = (rho_p * V) * h3;
  double tr = (Q[0][0] + Q[1][1]) + Q[2][2];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) I[a][b] = (rho_p * h3) * ((a == b ? tr : 0.0) - Q[a][b]);
}

/* params: rho_p, g[3], drive amplitude, drive period, drive direction[3],
 * kn, kt, eta_n, eta_t, mu, Rs, nsub, coupling.  Sets up every particle of
 * motion 3 (centre of mass as its centre, state at rest but for its initial
 * velocity); call after the particles are added and before seeding. */
int orc_set_dem(orc_domain* d, const double* prm) {
  d->rho_p = prm[0];
  for (int a = 0; a < 3; a++) {
    d->g[a] = prm[1 + a];
    d->drive_dir[a] = prm[6 + a];
  }
  d->drive_amp = prm[4];
  d->drive_period = prm[5];
  d->kn = prm[9];
  d->kt = prm[10];
  d->eta_n = prm[11];
  d->eta_t = prm[12];
  d->mu = prm[13];
  d->Rs = prm[14];
  d->nsub = (int)prm[15];
  d->coupling = (int)prm[16];
  if (d->nsub < 1 || !(d->rho_p > 0.0)) return -1;
  memset(d->xi, 0, sizeof(d->xi));
  memset(d->xiw, 0, sizeof(d->xiw));
  d->ndem = 0;
  for (int pi = 0; pi < d->np; pi++) {
    OPart* p = &d->P[pi];
    if (p->motion != 3) continue;
    double com[3], I[3][3];
    mass_properties(p, d->rho_p, &p->mass, com, I);
    for (int i = 0; i < p->nc; i++)
      for (int a = 0; a < 3; a++) p->b[3 * i + a] = p->b[3 * i + a] - com[a];
    double K = 0.0, bmax = 0.0;
    for (int i = 0; i < p->nc; i++) {
      K = K + p->k[i];
      const double* b = p->b + 3 * i;
      double r = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      if (r > bmax) bmax = r;
    }
    if (!(sqrt(K) > d->Rs)) return -1;
    p->rb = bmax + sqrt(K);
    p->cutsq = (p->rb + 2.0) * (p->rb + 2.0);
    p->cin = (sqrt(K) / (sqrt(K) - d->Rs)) * (sqrt(K) / (sqrt(K) - d->Rs));
    memcpy(p->Ib, I, sizeof(I));
    if (inv3(I, p->Ibinv) != 0) return -1;
    for (int a = 0; a < 3; a++) {
      p->c[a] = p->c0[a] + com[a];
      p->v[a] = p->vel[a];
      p->L[a] = 0.0;
      p->w[a] = 0.0;
    }
    p->q[0] = 1.0;
    p->q[1] = p->q[2] = p->q[3] = 0.0;
    p->wb[0] = (double*)malloc(sizeof(double) * 3 * p->nc);
    p->wb[1] = (double*)malloc(sizeof(double) * 3 * p->nc);
    rotate_offsets(p, p->q, p->wb[0]);
    rotate_offsets(p, p->q, p->wb[1]);
    memset(p->acc, 0, sizeof(p->acc));
    d->ndem++;
  }
  return 0;
}

/* Node nd's share of the hydrodynamic force on each coupled particle with a
 * solid fraction there (eps_p / sum eps of the exchange fx), and its torque
 * about the particle's centre; summed in fixed point (2^48), so that the
 * sums do not depend on the order of the nodes. */
static int64_t fix48(double x) { return (int64_t)llrint(x * ORC_FIX); }

static void dem_accumulate(orc_domain* d, const void* Pv, const int nd[3], const double* ep, double es,
                           const double fx[3]) {
  const Poses* Pt = (const Poses*)Pv;
  for (int p = 0; p < d->np; p++) {
    OPart* q = &d->P[p];
    if (q->motion != 3 || !(ep[p] > 0.0)) continue;
    double share = ep[p] / es;
    double F[3], dl[3];
    for (int a = 0; a < 3; a++) {
      F[a] = share * fx[a];
      dl[a] = rel(d, a, nd[a], Pt->c[p][a], 0.5);
    }
    double T[3] = {dl[1] * F[2] - dl[2] * F[1], dl[2] * F[0] - dl[0] * F[2], dl[0] * F[1] - dl[1] * F[0]};
    int64_t v[6] = {fix48(F[0]), fix48(F[1]), fix48(F[2]), fix48(T[0]), fix48(T[1]), fix48(T[2])};
    for (int k = 0; k < 6; k++) {
#pragma omp atomic
      q->acc[k] += v[k];
    }
  }
}

/* Hessian of M at offset dl: sum_i k_i (8 r r^T / |r|^6 - 2 I / |r|^4). */
static void mb_hess(const double* b, const double* k, int nc, const double dl[3], double H[3][3]) {
  for (int a = 0; a < 3; a++)
    for (int c = 0; c < 3; c++) H[a][c] = 0.0;
  for (int i = 0; i < nc; i++) {
    double r[3] = {dl[0] - b[3 * i], dl[1] - b[3 * i + 1], dl[2] - b[3 * i + 2]};
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double r4 = r2 * r2;
    double a8 = (8.0 * k[i]) / (r4 * r2), a2 = (2.0 * k[i]) / r4;
    for (int a = 0; a < 3; a++)
      for (int c = 0; c < 3; c++) H[a][c] = H[a][c] + (a8 * (r[a] * r[c]) - (a == c ? a2 : 0.0));
  }
}

static void solve3x3(const double A[3][3], const double b[3], double x[3], int* ok) {
  double X[3][3];
  if (inv3(A, X) != 0) {
    *ok = 0;
    return;
  }
  for (int a = 0; a < 3; a++) x[a] = (X[a][0] * b[0] + X[a][1] * b[1]) + X[a][2] * b[2];
  *ok = 1;
}

/* Eq. 8: the point of the inner body (level cin) reached from x along the
 * gradient, q from a first-order Taylor expansion.  The expansion is taken
 * in the field g = M^(-1/2), whose level sets are those of M and which is
 * r / sqrt(k) for one control point, so that the point is exact for a
 * sphere.  Returns 0 when x is inside the inner body. */
static int inner_point(const double* b, const double* k, int nc, double cin, const double x[3], double xc[3]) {
  double M = mb_Mb(b, k, nc, x);
  if (!(M < cin)) return 0;
  double gm[3];
  mb_gradb(b, k, nc, x, gm);
  double g = 1.0 / sqrt(M), gin = 1.0 / sqrt(cin);
  double s = -0.5 * (g / M); /* dg/dM = -M^(-3/2) / 2 */
  double gg[3] = {s * gm[0], s * gm[1], s * gm[2]};
  double n2 = (gg[0] * gg[0] + gg[1] * gg[1]) + gg[2] * gg[2];
  if (!(n2 > 0.0)) return 0;
  double q = (gin - g) / n2;
  for (int a = 0; a < 3; a++) xc[a] = x[a] + q * gg[a];
  return 1;
}

/* Contact between coupled particles i and j (Eq. 6-9): the minimum x_m of
 * M_i + M_j between them by Newton-Raphson (start: the midpoint of the
 * centres, j's as the minimum image seen from i; 40 iterations at most,
 * stop when the step is below 1e-12), the closest points of the inner
 * bodies (Eq. 8, inner_point), the normal from i's point to j's and the
 * overlap of the dilation spheres (Eq. 9).
 * Returns 1 with (xcp offset from c_i, n, delta) when they overlap. */
static int contact_pair(const orc_domain* d, int i, int j, const double ci[3], const double cj[3], const double* bi,
                        const double* bj, double xcp[3], double n[3], double* delta) {
  const OPart* P = &d->P[i];
  const OPart* Q = &d->P[j];
  double dc[3];
  for (int a = 0; a < 3; a++) {
    dc[a] = cj[a] - ci[a];
    if (!d->bc[a]) {
      double L = (double)d->n[a];
      dc[a] = dc[a] - L * floor(dc[a] / L + 0.5);
    }
  }
  double r2 = dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2];
  double rr = P->rb + Q->rb;
  if (!(r2 < rr * rr)) return 0;
  double x[3] = {0.5 * dc[0], 0.5 * dc[1], 0.5 * dc[2]}; /* offset from c_i */
  for (int it = 0; it < 40; it++) {
    double xj[3] = {x[0] - dc[0], x[1] - dc[1], x[2] - dc[2]};
    double gi[3], gj[3], Hi[3][3], Hj[3][3], H[3][3], g[3], st[3];
    mb_gradb(bi, P->k, P->nc, x, gi);
    mb_gradb(bj, Q->k, Q->nc, xj, gj);
    mb_hess(bi, P->k, P->nc, x, Hi);
    mb_hess(bj, Q->k, Q->nc, xj, Hj);
    for (int a = 0; a < 3; a++) {
      g[a] = gi[a] + gj[a];
      for (int c = 0; c < 3; c++) H[a][c] = Hi[a][c] + Hj[a][c];
    }
    int ok;
    solve3x3(H, g, st, &ok);
    if (!ok || !(isfinite(st[0]) && isfinite(st[1]) && isfinite(st[2]))) return 0;
    for (int a = 0; a < 3; a++) x[a] = x[a] - st[a];
    double sn = sqrt(st[0] * st[0] + st[1] * st[1] + st[2] * st[2]);
    if (sn < 1e-12) break;
  }
  double xj[3] = {x[0] - dc[0], x[1] - dc[1], x[2] - dc[2]};
  double x0[3], x1[3], dd[3];
  if (!inner_point(bi, P->k, P->nc, P->cin, x, x0)) return 0;
  if (!inner_point(bj, Q->k, Q->nc, Q->cin, xj, x1)) return 0;
  for (int a = 0; a < 3; a++) {
    x1[a] = x1[a] + dc[a];
    dd[a] = x1[a] - x0[a];
  }
  double dist = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  double del = (d->Rs + d->Rs) - dist;
  if (!(del > 0.0) || !(dist > 0.0)) return 0;
  for (int a = 0; a < 3; a++) {
    n[a] = dd[a] / dist;
    xcp[a] = x0[a] + (d->Rs - 0.5 * del) * n[a];
  }
  *delta = del;
  return 1;
}

/* Contact of coupled particle i with the wall plane of wall axis `ax` on
 * side `side` (Eq. 10-11): the point of the inner metaball whose gradient is
 * normal to the wall, by Newton-Raphson on (grad M tangential = 0,
 * M = cin) from the inner surface point on the ray from the centre towards
 * the wall; n points from the particle to the wall.  Returns 1 with (xcp
 * offset from c_i, n, delta) when the dilation sphere crosses the plane. */
static int contact_wall(const orc_domain* d, int i, const double ci[3], const double* bi, int ax, int side,
                        double xcp[3], double n[3], double* delta) {
  const OPart* P = &d->P[i];
  double plane = side ? (double)(d->n[ax] - 1) : 1.0;
  double gap = side ? plane - ci[ax] : ci[ax] - plane; /* distance from the centre to the plane */
  if (!(gap < P->rb + d->Rs)) return 0;
  int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
  double dir = side ? 1.0 : -1.0;
  double x[3] = {0.0, 0.0, 0.0};
  /* start: bisection for M = cin on the ray from the centre towards the wall */
  double lo = 0.0, hi = P->rb;
  for (int it = 0; it < 60; it++) {
    double m = 0.5 * (lo + hi);
    double y[3] = {0.0, 0.0, 0.0};
    y[ax] = dir * m;
    if (mb_Mb(bi, P->k, P->nc, y) >= P->cin) lo = m;
    else hi = m;
  }
  x[ax] = dir * lo;
  for (int it = 0; it < 40; it++) {
    double g[3], H[3][3], J[3][3], r[3], st[3];
    mb_gradb(bi, P->k, P->nc, x, g);
    mb_hess(bi, P->k, P->nc, x, H);
    double M = mb_Mb(bi, P->k, P->nc, x);
    r[0] = g[t1];
    r[1] = g[t2];
    r[2] = M - P->cin;
    for (int c = 0; c < 3; c++) {
      J[0][c] = H[t1][c];
      J[1][c] = H[t2][c];
      J[2][c] = g[c];
    }
    int ok;
    solve3x3(J, r, st, &ok);
    if (!ok || !(isfinite(st[0]) && isfinite(st[1]) && isfinite(st[2]))) return 0;
    for (int a = 0; a < 3; a++) x[a] = x[a] - st[a];
    double sn = sqrt(st[0] * st[0] + st[1] * st[1] + st[2] * st[2]);
    if (sn < 1e-12) break;
  }
  double dist = side ? plane - (ci[ax] + x[ax]) : (ci[ax] + x[ax]) - plane;
  double del = d->Rs - dist;
  if (!(del > 0.0)) return 0;
  for (int a = 0; a < 3; a++) n[a] = 0.0;
  n[ax] = dir;
  for (int a = 0; a < 3; a++) xcp[a] = x[a] + (d->Rs - 0.5 * del) * n[a];
  *delta = del;
  return 1;
}

static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Spring-dashpot force (Eq. 5) on body B from body A at a contact: normal n
 * from A to B, overlap delta, relative velocity vr = v_B - v_A at the contact
 * point, tangential spring xi (updated).  Returns the force on B. */
static void contact_force(const orc_domain* d, const double n[3], double delta, const double vr[3], double dt,
                          double xi[3], double F[3]) {
  double vn = (vr[0] * n[0] + vr[1] * n[1]) + vr[2] * n[2];
  double Fn = d->kn * delta - d->eta_n * vn;
  if (Fn < 0.0) Fn = 0.0;
  double vt[3];
  for (int a = 0; a < 3; a++) vt[a] = vr[a] - vn * n[a];
  for (int a = 0; a < 3; a++) xi[a] = xi[a] + vt[a] * dt;
  double xn = (xi[0] * n[0] + xi[1] * n[1]) + xi[2] * n[2];
  for (int a = 0; a < 3; a++) xi[a] = xi[a] - xn * n[a];
  double Ft[3];
  for (int a = 0; a < 3; a++) Ft[a] = -(d->kt * xi[a]) - d->eta_t * vt[a];
  double ft = sqrt((Ft[0] * Ft[0] + Ft[1] * Ft[1]) + Ft[2] * Ft[2]);
  double cap = d->mu * Fn;
  if (ft > cap) {
    for (int a = 0; a < 3; a++) {
      Ft[a] = Ft[a] * (cap / ft);
      /* the spring stretched to what the capped force needs (none without a spring) */
      xi[a] = d->kt > 0.0 ? -(Ft[a] + d->eta_t * vt[a]) / d->kt : 0.0;
    }
  }
  for (int a = 0; a < 3; a++) F[a] = Fn * n[a] + Ft[a];
}

/* Advance every coupled particle by one fluid step (nsub substeps) from the
 * state at t, with the hydrodynamic force of the fluid update of t. */
static void dem_advance(orc_domain* d) {
  const double dt = 1.0 / (double)d->nsub;
  for (int p = 0; p < d->np; p++) {
    OPart* q = &d->P[p];
    if (q->motion != 3) continue;
    for (int a = 0; a < 3; a++) {
      q->Fh[a] = d->coupling ? (double)q->acc[a] / ORC_FIX : 0.0;
      q->Th[a] = d->coupling ? (double)q->acc[3 + a] / ORC_FIX : 0.0;
    }
    memset(q->acc, 0, sizeof(q->acc));
  }
  for (int s = 0; s < d->nsub; s++) {
    double tau = (double)d->t + (double)s * dt;
    double F[ORC_MAXP][3], T[ORC_MAXP][3];
    double ph = tau / d->drive_period;
    ph = ph - floor(ph);
    double sn, cs;
    sincos2pi(ph, &sn, &cs);
    for (int p = 0; p < d->np; p++) {
      OPart* q = &d->P[p];
      if (q->motion != 3) continue;
      for (int a = 0; a < 3; a++) {
        F[p][a] = (q->mass * d->g[a] + q->mass * ((d->drive_amp * cs) * d->drive_dir[a])) + q->Fh[a];
        T[p][a] = q->Th[a];
      }
    }
    /* particle pairs */
    for (int i = 0; i < d->np; i++) {
      if (d->P[i].motion != 3) continue;
      for (int j = i + 1; j < d->np; j++) {
        if (d->P[j].motion != 3) continue;
        OPart *A = &d->P[i], *Bq = &d->P[j];
        double xcp[3], n[3], del;
        if (!contact_pair(d, i, j, A->c, Bq->c, A->wb[0], Bq->wb[0], xcp, n, &del)) {
          memset(d->xi[i][j], 0, sizeof(d->xi[i][j]));
          continue;
        }
        /* offsets of the contact point from both centres (j's via the minimum image) */
        double dc[3], rj[3], va[3], vb[3], wa[3], wb[3], vr[3], Fc[3];
        for (int a = 0; a < 3; a++) {
          dc[a] = Bq->c[a] - A->c[a];
          if (!d->bc[a]) {
            double L = (double)d->n[a];
            dc[a] = dc[a] - L * floor(dc[a] / L + 0.5);
          }
          rj[a] = xcp[a] - dc[a];
        }
        cross3(A->w, xcp, wa);
        cross3(Bq->w, rj, wb);
        for (int a = 0; a < 3; a++) {
          va[a] = A->v[a] + wa[a];
          vb[a] = Bq->v[a] + wb[a];
          vr[a] = vb[a] - va[a];
        }
        contact_force(d, n, del, vr, dt, d->xi[i][j], Fc);
        double ta[3], tb[3], mF[3] = {-Fc[0], -Fc[1], -Fc[2]};
        cross3(rj, Fc, tb);
        cross3(xcp, mF, ta);
        for (int a = 0; a < 3; a++) {
          F[j][a] = F[j][a] + Fc[a];
          T[j][a] = T[j][a] + tb[a];
          F[i][a] = F[i][a] + mF[a];
          T[i][a] = T[i][a] + ta[a];
        }
      }
    }
    /* walls */
    for (int i = 0; i < d->np; i++) {
      OPart* A = &d->P[i];
      if (A->motion != 3) continue;
      for (int ax = 0; ax < 3; ax++) {
        if (!d->bc[ax]) continue;
        for (int side = 0; side < 2; side++) {
          double xcp[3], n[3], del;
          double* xi = d->xiw[i][2 * ax + side];
          if (!contact_wall(d, i, A->c, A->wb[0], ax, side, xcp, n, &del)) {
            memset(xi, 0, sizeof(double) * 3);
            continue;
          }
          double wa[3], vr[3], Fc[3];
          cross3(A->w, xcp, wa);
          for (int a = 0; a < 3; a++) vr[a] = d->wu[ax][side][a] - (A->v[a] + wa[a]);
          contact_force(d, n, del, vr, dt, xi, Fc);
          double mF[3] = {-Fc[0], -Fc[1], -Fc[2]}, ta[3];
          cross3(xcp, mF, ta);
          for (int a = 0; a < 3; a++) {
            F[i][a] = F[i][a] + mF[a];
            T[i][a] = T[i][a] + ta[a];
          }
        }
      }
    }
    /* Newton-Euler, symplectic Euler */
    for (int p = 0; p < d->np; p++) {
      OPart* q = &d->P[p];
      if (q->motion != 3) continue;
      for (int a = 0; a < 3; a++) {
        q->v[a] = q->v[a] + (F[p][a] / q->mass) * dt;
        q->c[a] = q->c[a] + q->v[a] * dt;
        q->L[a] = q->L[a] + T[p][a] * dt;
      }
      if (!d->bc[0] || !d->bc[1] || !d->bc[2])
        for (int a = 0; a < 3; a++)
          if (!d->bc[a]) {
            double L = (double)d->n[a];
            q->c[a] = q->c[a] - L * floor(q->c[a] / L);
          }
      /* w = R Ib^-1 R^T L */
      double R[3][3], y[3], z[3];
      quat_R(q->q, R);
      for (int a = 0; a < 3; a++) y[a] = (R[0][a] * q->L[0] + R[1][a] * q->L[1]) + R[2][a] * q->L[2];
      for (int a = 0; a < 3; a++) z[a] = (q->Ibinv[a][0] * y[0] + q->Ibinv[a][1] * y[1]) + q->Ibinv[a][2] * y[2];
      for (int a = 0; a < 3; a++) q->w[a] = (R[a][0] * z[0] + R[a][1] * z[1]) + R[a][2] * z[2];
      /* q += dt/2 (0, w) q, normalised */
      double w0 = q->q[0], w1 = q->q[1], w2 = q->q[2], w3 = q->q[3];
      double hw[3] = {0.5 * dt * q->w[0], 0.5 * dt * q->w[1], 0.5 * dt * q->w[2]};
      double n0 = w0 - ((hw[0] * w1 + hw[1] * w2) + hw[2] * w3);
      double n1 = w1 + ((hw[0] * w0 + hw[1] * w3) - hw[2] * w2);
      double n2 = w2 + ((hw[1] * w0 + hw[2] * w1) - hw[0] * w3);
      double n3 = w3 + ((hw[2] * w0 + hw[0] * w2) - hw[1] * w1);
      double nn = sqrt(((n0 * n0 + n1 * n1) + n2 * n2) + n3 * n3);
      q->q[0] = n0 / nn;
      q->q[1] = n1 / nn;
      q->q[2] = n2 / nn;
      q->q[3] = n3 / nn;
      rotate_offsets(q, q->q, q->wb[0]);
    }
  }
}

/* One coupled step t -> t+1: fluid at P(t) (its momentum exchange gives the
 * hydrodynamic force on the coupled particles), the coupled particles
 * advanced to t+1, walkers with u(t) against P(t+1). */
void orc_step(orc_domain* d, int nsteps) {
  for (int s = 0; s < nsteps; s++) {
    Poses Pt, Pn;
    all_poses(d, d->t, &Pt);
    if (d->ndem > 0) {
      /* Pt points at the offsets of the current orientation; keep a copy,
       * since the particle update rotates them */
      for (int p = 0; p < d->np; p++)
        if (d->P[p].motion == 3) {
          memcpy(d->P[p].wb[1], d->P[p].wb[0], sizeof(double) * 3 * d->P[p].nc);
          Pt.b[p] = d->P[p].wb[1];
        }
    }
    if (d->ibb && d->ndem > 0)
      /* the exchange of the streaming that delivered f(t) drives the update t -> t+1 */
      for (int p = 0; p < d->np; p++)
        if (d->P[p].motion == 3) {
          memcpy(d->P[p].acc, d->P[p].acc_ibb, sizeof(d->P[p].acc));
          memset(d->P[p].acc_ibb, 0, sizeof(d->P[p].acc_ibb));
        }
    fluid_step(d, &Pt);
    if (d->ndem > 0) dem_advance(d);
    all_poses(d, d->t + 1, &Pn);
    if (d->nw) walkers_step(d, &Pn);
    d->t++;
  }
}

/* ----------------------------------------------------------- seeding */
/* kind 0 uniform over the fluid box, 1 Gaussian (centre, sigma), 2 band along
 * one axis, 3 explicit positions.  Attempt a of walker w draws Philox counter
 * (w, 0xFFFFFFFF, 16 + a, 0); positions inside a particle at P(0) or outside
 * the fluid range of a wall axis are rejected and redrawn.  remove_inside = 1
 * instead drops such walkers after one draw (the paper's removal at the first
 * step) and renumbers the survivors in order.  Returns the number placed, or
 * -1 if a walker exhausted its attempts. */
int64_t orc_seed(orc_domain* d, int kind, const double centre[3], double sigma, int band_axis,
                 double band_lo, double band_hi, const double* xyz, int64_t n, int max_attempts,
                 int remove_inside, const double ref[3]) {
  Poses P0;
  all_poses(d, 0, &P0);
  free(d->cell); free(d->off); free(d->img);
  d->cell = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  d->off = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
  d->img = (int32_t*)calloc(3 * (n > 0 ? n : 1), sizeof(int32_t));
  double* tmp = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
  int32_t* tcell = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  unsigned char* okv = (unsigned char*)calloc(n > 0 ? n : 1, 1);
  int attempts = remove_inside ? 1 : max_attempts;
  if (kind == 3) attempts = 1;
  int fail = 0;
#pragma omp parallel for schedule(static) reduction(| : fail)
  for (int64_t w = 0; w < n; w++) {
    int placed = 0;
    for (int at = 0; at < attempts && !placed; at++) {
      double X[3];
      if (kind == 3) {
        for (int a = 0; a < 3; a++) X[a] = xyz[3 * w + a];
      } else {
        uint32_t ctr[4] = {(uint32_t)w, 0xFFFFFFFFu, 16u + (uint32_t)at, 0u}, r[4];
        philox(ctr, d->key, r);
        if (kind == 1) {
          double z[3];
          normals3(r, z);
          for (int a = 0; a < 3; a++) X[a] = centre[a] + sigma * z[a];
        } else {
          for (int a = 0; a < 3; a++) {
            double lo = d->bc[a] ? 1.0 : 0.0, hi = d->bc[a] ? (double)(d->n[a] - 1) : (double)d->n[a];
            if (kind == 2 && a == band_axis) { lo = band_lo; hi = band_hi; }
            X[a] = lo + u01(r[a]) * (hi - lo);
          }
        }
      }
      int cell[3], okp = 1;
      double o[3];
      for (int a = 0; a < 3; a++) {
        double L = (double)d->n[a];
        double x = X[a];
        if (!d->bc[a]) {
          x = x - L * floor(x / L);
          if (x >= L) x = 0.0;
        } else if (x < 1.0 || x >= L - 1.0) {
          okp = 0;
        }
        double k = floor(x);
        cell[a] = (int)k;
        o[a] = x - k;
      }
      if (!okp) continue;
      if (inside_any(d, &P0, cell, o) >= 0) continue;
      tcell[w] = (int32_t)nidx(d, cell[0], cell[1], cell[2]);
      for (int a = 0; a < 3; a++) tmp[3 * w + a] = o[a];
      placed = 1;
    }
    okv[w] = (unsigned char)placed;
    if (!placed && !remove_inside) fail = 1;
  }
  int64_t m = 0;
  for (int64_t w = 0; w < n; w++) {
    if (!okv[w]) continue;
    d->cell[m] = tcell[w];
    m++;
  }
  /* offsets in SoA order */
  double* off = d->off;
  int64_t k = 0;
  for (int64_t w = 0; w < n; w++) {
    if (!okv[w]) continue;
    for (int a = 0; a < 3; a++) off[a * m + k] = tmp[3 * w + a];
    k++;
  }
  free(tmp); free(tcell); free(okv);
  d->nw = m;
  for (int a = 0; a < 3; a++) d->ref[a] = ref[a];
  d->seeded = 1;
  if (fail) return -1;
  return m;
}

/* ----------------------------------------------------------- reports */
/* Eq. 16: n_s = number of walkers whose cell is the node. */
void orc_occupancy(const orc_domain* d, uint32_t* ns) {
  memset(ns, 0, sizeof(uint32_t) * d->N);
  for (int64_t w = 0; w < d->nw; w++) ns[d->cell[w]]++;
}

/* Concentration profile along an axis (Eq. 16 summed over the other two
 * axes): walkers per layer of the lattice along `axis`. */
void orc_profile(const orc_domain* d, int axis, uint64_t* counts) {
  const int nx = d->n[0], ny = d->n[1];
  memset(counts, 0, sizeof(uint64_t) * d->n[axis]);
  for (int64_t w = 0; w < d->nw; w++) {
    int32_t lc = d->cell[w];
    int c[3] = {lc % nx, (lc / nx) % ny, lc / (nx * ny)};
    counts[c[axis]]++;
  }
}

/* Moments (sequential sums in index order):
 * out[0]   walker count
 * out[1-3] sum (X - ref), X unwrapped with image counts
 * out[4-6] sum (X - ref)^2
 * out[7]   sum rho over fluid nodes       out[8-10] sum rho u over fluid nodes
 * out[11-13] sum (1-eps) u / sum (1-eps)  (fluid-volume average)
 * out[14-16] sum eps us / sum eps         (particle-volume average; 0 if none)
 * out[17]  sum eps                        out[18] step */
void orc_moments(const orc_domain* d, double* out) {
  const int64_t N = d->N, nw = d->nw;
  const int nx = d->n[0], ny = d->n[1];
  memset(out, 0, sizeof(double) * 19);
  out[0] = (double)nw;
  for (int64_t w = 0; w < nw; w++) {
    int32_t lc = d->cell[w];
    int cell[3] = {lc % nx, (lc / nx) % ny, lc / (nx * ny)};
    for (int a = 0; a < 3; a++) {
      int64_t X = (int64_t)cell[a] + (int64_t)d->img[a * nw + w] * (int64_t)d->n[a];
      double dv = ((double)X - d->ref[a]) + d->off[a * nw + w];
      out[1 + a] = out[1 + a] + dv;
      out[4 + a] = out[4 + a] + dv * dv;
    }
  }
  double s1e = 0.0, se = 0.0, fu[3] = {0, 0, 0}, pv[3] = {0, 0, 0};
  for (int64_t id = 0; id < N; id++) {
    if (d->wall[id]) continue;
    double r = d->rho[id], e = d->eps[id];
    out[7] = out[7] + r;
    for (int a = 0; a < 3; a++) {
      double ua = d->u[a * N + id];
      out[8 + a] = out[8 + a] + r * ua;
      fu[a] = fu[a] + (1.0 - e) * ua;
      pv[a] = pv[a] + e * d->us[a * N + id];
    }
    s1e = s1e + (1.0 - e);
    se = se + e;
  }
  for (int a = 0; a < 3; a++) {
    out[11 + a] = s1e > 0.0 ? fu[a] / s1e : 0.0;
    out[14 + a] = se > 0.0 ? pv[a] / se : 0.0;
  }
  out[17] = se;
  out[18] = (double)d->t;
}

/* ----------------------------------------------------------- accessors */
int64_t orc_num_nodes(const orc_domain* d) { return d->N; }
int64_t orc_num_walkers(const orc_domain* d) { return d->nw; }
int64_t orc_time(const orc_domain* d) { return d->t; }
void orc_get_ref(const orc_domain* d, double ref[3]) { memcpy(ref, d->ref, sizeof(d->ref)); }
void orc_counters(const orc_domain* d, uint64_t* c) { memcpy(c, d->cnt, sizeof(d->cnt)); }
void orc_get_f(const orc_domain* d, double* f) { memcpy(f, d->f, sizeof(double) * 19 * d->N); }
void orc_set_f(orc_domain* d, const double* f) { memcpy(d->f, f, sizeof(double) * 19 * d->N); }
void orc_get_fields(const orc_domain* d, double* rho, double* u, double* eps, double* us) {
  if (rho) memcpy(rho, d->rho, sizeof(double) * d->N);
  if (u) memcpy(u, d->u, sizeof(double) * 3 * d->N);
  if (eps) memcpy(eps, d->eps, sizeof(double) * d->N);
  if (us) memcpy(us, d->us, sizeof(double) * 3 * d->N);
}
void orc_get_walkers(const orc_domain* d, int32_t* cell, double* off, int32_t* img) {
  if (cell) memcpy(cell, d->cell, sizeof(int32_t) * d->nw);
  if (off) memcpy(off, d->off, sizeof(double) * 3 * d->nw);
  if (img) memcpy(img, d->img, sizeof(int32_t) * 3 * d->nw);
}
/* Replace the walker set (positions as cell index + offset); for tests. */
void orc_set_walkers(orc_domain* d, int64_t nw, const int32_t* cell, const double* off,
                     const double ref[3]) {
  free(d->cell); free(d->off); free(d->img);
  d->nw = nw;
  d->cell = (int32_t*)malloc(sizeof(int32_t) * (nw > 0 ? nw : 1));
  d->off = (double*)malloc(sizeof(double) * 3 * (nw > 0 ? nw : 1));
  d->img = (int32_t*)calloc(3 * (nw > 0 ? nw : 1), sizeof(int32_t));
  memcpy(d->cell, cell, sizeof(int32_t) * nw);
  memcpy(d->off, off, sizeof(double) * 3 * nw);
  for (int a = 0; a < 3; a++) d->ref[a] = ref[a];
}

/* Threads of the OpenMP loops (the CPU-baseline timing runs 1 and all). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------ exported pieces for the pins */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox(ctr, key, out); }
double orc_ln_export(double u) { return orc_ln(u); }
void orc_sincos2pi(double u, double* s, double* c) { sincos2pi(u, s, c); }
void orc_normals(const uint32_t ctr[4], const uint32_t key[2], double z[3]) {
  uint32_t r[4];
  philox(ctr, key, r);
  normals3(r, z);
}
/* normals for counters (id, t, purpose, 0), id = 0..n-1 */
void orc_normals_batch(uint32_t t, uint32_t purpose, const uint32_t key[2], int64_t n, double* z) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    uint32_t ctr[4] = {(uint32_t)i, t, purpose, 0u}, r[4];
    philox(ctr, key, r);
    normals3(r, z + 3 * i);
  }
}
void orc_feq(double rho, const double u[3], double out[19]) {
  init_weights();
  for (int i = 0; i < 19; i++) out[i] = feq(i, rho, u);
}
void orc_lattice(int32_t e[57], double w[19]) {
  init_weights();
  for (int i = 0; i < 19; i++) {
    w[i] = WT[i];
    for (int a = 0; a < 3; a++) e[3 * i + a] = EV[i][a];
  }
}
void orc_collide_node(orc_domain* d, const double f[19], double eps, const double us[3],
                      double out[19], double* rho, double u[3]) {
  collide_node(d, f, eps, us, out, rho, u);
}
double orc_particle_M(const orc_domain* d, int p, int64_t t, const int cell[3], const double x[3]) {
  Poses P;
  all_poses(d, t, &P);
  return M_at(d, &P, p, cell, x);
}
void orc_particle_grad(const orc_domain* d, int p, int64_t t, const int cell[3], const double x[3],
                       double g[3]) {
  Poses P;
  all_poses(d, t, &P);
  double dl[3];
  delta_to(d, &P, p, cell, x, dl);
  grad_at(d, &P, p, dl, g);
}
void orc_particle_pose(const orc_domain* d, int p, int64_t t, double c[3], double v[3]) {
  if (d->P[p].motion == 3) {
    memcpy(c, d->P[p].c, sizeof(double) * 3);
    memcpy(v, d->P[p].v, sizeof(double) * 3);
    return;
  }
  pose(&d->P[p], t, c, v);
}
/* State of coupled particle p: c[3], v[3], q[4], L[3], w[3], Fh[3], Th[3],
 * mass, Ib[9] (27 doubles). */
void orc_dem_state(const orc_domain* d, int p, double* out) {
  const OPart* q = &d->P[p];
  memcpy(out, q->c, 24);
  memcpy(out + 3, q->v, 24);
  memcpy(out + 6, q->q, 32);
  memcpy(out + 10, q->L, 24);
  memcpy(out + 13, q->w, 24);
  memcpy(out + 16, q->Fh, 24);
  memcpy(out + 19, q->Th, 24);
  out[22] = q->mass;
  for (int a = 0; a < 3; a++)
    for (int c = 0; c < 3; c++) out[23 + 3 * a + c] = q->Ib[a][c];
}
/* Overwrite a coupled particle's velocity and angular momentum (test set-up). */
void orc_dem_set_motion(orc_domain* d, int p, const double v[3], const double L[3]) {
  OPart* q = &d->P[p];
  memcpy(q->v, v, 24);
  memcpy(q->L, L, 24);
  double R[3][3], y[3], z[3];
  quat_R(q->q, R);
  for (int a = 0; a < 3; a++) y[a] = (R[0][a] * q->L[0] + R[1][a] * q->L[1]) + R[2][a] * q->L[2];
  for (int a = 0; a < 3; a++) z[a] = (q->Ibinv[a][0] * y[0] + q->Ibinv[a][1] * y[1]) + q->Ibinv[a][2] * y[2];
  for (int a = 0; a < 3; a++) q->w[a] = (R[a][0] * z[0] + R[a][1] * z[1]) + R[a][2] * z[2];
}
double orc_particle_rb(const orc_domain* d, int p) { return d->P[p].rb; }
/* Algorithm 1 on a caller-given segment; returns iterations used encoded as
 * success flag in *ok. */
double orc_bisect_segment(const orc_domain* d, int p, int64_t t, const int cell[3], const double a0[3],
                          const double dir[3], double s_out, double s_in, int imax, int* ok) {
  Poses P;
  all_poses(d, t, &P);
  double s = -1.0;
  *ok = bisect(d, &P, p, cell, a0, dir, s_out, s_in, imax, &s);
  return s;
}
/* Eq. 19 with the normal normalised: t_r = t_i - 2 (t_i . n) n. */
void orc_reflect(const double ti[3], const double g[3], double tr[3]) {
  double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  double nv[3];
  for (int a = 0; a < 3; a++) nv[a] = g[a] / gn;
  double dt = ti[0] * nv[0] + ti[1] * nv[1] + ti[2] * nv[2];
  for (int a = 0; a < 3; a++) tr[a] = ti[a] - (2.0 * dt) * nv[a];
}

/* Eq. 38-40: sigma^2/(2R)^2 = K (U_slip / 2R) t + offset fitted by ordinary
 * least squares (normal equations) on samples i0..n-1, then D_alpha =
 * K / (1 - phi).  Returns 0 on success. */
int orc_dispersion_fit(const double* t, const double* sigma2, int n, int i0, double two_r, double u_slip,
                       double phi, double* K, double* D_alpha) {
  if (n - i0 < 2 || u_slip == 0.0 || phi >= 1.0) return -1;
  double S = 0, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0;
  for (int i = i0; i < n; i++) {
    double y = sigma2[i] / (two_r * two_r);
    S += 1.0;
    Sx += t[i];
    Sy += y;
    Sxx += t[i] * t[i];
    Sxy += t[i] * y;
  }
  double den = S * Sxx - Sx * Sx;
  if (den == 0.0) return -1;
  double slope = (S * Sxy - Sx * Sy) / den;
  *K = slope / (u_slip / two_r);
  *D_alpha = *K / (1.0 - phi);
  return 0;
}

/* The dispersion pipeline of Sec. 4 from a series of n moment records
 * (orc_moments layout, 19 doubles each):
 *   variance along the dispersion axis: sumsq/N - (sum/N)^2 per sample;
 *   Eq. 39: the slip velocity is the gap between the maxima over time of the
 *   fluid-average and the particle-average velocity along the flow axis
 *   (taken as a magnitude);
 *   solid fraction: the solid volume averaged over the samples after the
 *   first step, over the node count;
 *   Eq. 38 and 40 through orc_dispersion_fit on samples i0..n-1.
 * out5 = {u_slip, phi, K, D_alpha, intercept of the line}.  Returns 0 on
 * success. */
int orc_dispersion_from_moments(const double* mom, int n, int i0, int disp_axis, int flow_axis, double n_nodes,
                                double two_r, double* sigma2, double* out5) {
  if (n - i0 < 2 || disp_axis < 0 || disp_axis > 2 || flow_axis < 0 || flow_axis > 2 || !(n_nodes > 0.0))
    return -1;
  double* t = (double*)malloc(sizeof(double) * n);
  double* v = (double*)malloc(sizeof(double) * n);
  double umax = -INFINITY, pmax = -INFINITY, solid = 0.0;
  int ns = 0;
  for (int i = 0; i < n; i++) {
    const double* m = mom + 19 * i;
    double N = m[0];
    if (!(N > 0.0)) {
      free(t);
      free(v);
      return -1;
    }
    double mean = m[1 + disp_axis] / N;
    v[i] = m[4 + disp_axis] / N - mean * mean;
    t[i] = m[18];
    if (m[11 + flow_axis] > umax) umax = m[11 + flow_axis];
    if (m[14 + flow_axis] > pmax) pmax = m[14 + flow_axis];
    if (m[18] > 0.0) {
      solid = solid + m[17];
      ns = ns + 1;
    }
  }
  if (sigma2) memcpy(sigma2, v, sizeof(double) * n);
  double u_slip = fabs(umax - pmax);
  double phi = ns > 0 ? (solid / (double)ns) / n_nodes : 0.0;
  double K = 0.0, Da = 0.0;
  int r = orc_dispersion_fit(t, v, n, i0, two_r, u_slip, phi, &K, &Da);
  /* intercept of the least-squares line of sigma^2/(2R)^2 against t */
  double S = 0, Sx = 0, Sy = 0;
  for (int i = i0; i < n; i++) {
    S += 1.0;
    Sx += t[i];
    Sy += v[i] / (two_r * two_r);
  }
  double slope = K * (u_slip / two_r);
  out5[0] = u_slip;
  out5[1] = phi;
  out5[2] = K;
  out5[3] = Da;
  out5[4] = (Sy - slope * Sx) / S;
  free(t);
  free(v);
  return r;
}

/* Least-squares Gaussian y = A exp(-(x - mu)^2 / (2 s2)) through the points
 * (x_k, y_k), the profile fit of Sec. 4.  Gauss-Newton on (A, mu, s2) from
 * the moment estimates (weights y_k), each step solving the 3x3 normal
 * equations by Cramer's rule, halving the step while the residual sum of
 * squares does not decrease; stops when the relative change of every
 * parameter is below 1e-13 or after 200 steps.  out3 = {A, mu, s2}.
 * Returns 0, or -1 if fewer than 3 points are positive (three parameters
 * are not fixed by fewer) or the normal matrix is singular. */
static double gauss_rss(const double* x, const double* y, int n, const double p[3]) {
  double r = 0.0;
  for (int k = 0; k < n; k++) {
    double d = x[k] - p[1];
    double e = y[k] - p[0] * exp(-(d * d) / (2.0 * p[2]));
    r = r + e * e;
  }
  return r;
}

static double det3(const double m[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

int orc_gaussian_fit(const double* x, const double* y, int n, double* out3) {
  if (n < 3) return -1;
  double sw = 0.0, sx = 0.0, ymax = 0.0;
  int npos = 0;
  for (int k = 0; k < n; k++) {
    if (y[k] > 0.0) {
      sw = sw + y[k];
      sx = sx + y[k] * x[k];
      npos = npos + 1;
    }
    if (y[k] > ymax) ymax = y[k];
  }
  if (npos < 3) return -1;
  double p[3];
  p[1] = sx / sw;
  double sv = 0.0;
  for (int k = 0; k < n; k++)
    if (y[k] > 0.0) sv = sv + y[k] * (x[k] - p[1]) * (x[k] - p[1]);
  p[2] = sv / sw;
  if (!(p[2] > 0.0)) p[2] = 1.0;
  p[0] = ymax;
  double rss = gauss_rss(x, y, n, p);
  for (int it = 0; it < 200; it++) {
    double JtJ[3][3] = {{0}}, Jtr[3] = {0};
    for (int k = 0; k < n; k++) {
      double d = x[k] - p[1];
      double g = exp(-(d * d) / (2.0 * p[2]));
      double J[3] = {g, p[0] * g * d / p[2], p[0] * g * d * d / (2.0 * p[2] * p[2])};
      double r = y[k] - p[0] * g;
      for (int a = 0; a < 3; a++) {
        Jtr[a] = Jtr[a] + J[a] * r;
        for (int b = 0; b < 3; b++) JtJ[a][b] = JtJ[a][b] + J[a] * J[b];
      }
    }
    double D = det3(JtJ);
    if (D == 0.0 || !isfinite(D)) return -1;
    double step[3];
    for (int c = 0; c < 3; c++) {
      double M[3][3];
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) M[a][b] = b == c ? Jtr[a] : JtJ[a][b];
      step[c] = det3(M) / D;
    }
    double lam = 1.0, q[3], rq = 0.0;
    int ok = 0;
    for (int h = 0; h < 60; h++) {
      for (int a = 0; a < 3; a++) q[a] = p[a] + lam * step[a];
      if (q[2] > 0.0) {
        rq = gauss_rss(x, y, n, q);
        if (rq <= rss) {
          ok = 1;
          break;
        }
      }
      lam = 0.5 * lam;
    }
    if (!ok) break;
    double ch = 0.0;
    for (int a = 0; a < 3; a++) {
      double c = fabs(q[a] - p[a]) / (fabs(q[a]) > 1e-300 ? fabs(q[a]) : 1e-300);
      if (c > ch) ch = c;
      p[a] = q[a];
    }
    rss = rq;
    if (ch < 1e-13) break;
  }
  for (int a = 0; a < 3; a++) out3[a] = p[a];
  return 0;
}
