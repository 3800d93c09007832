/*
 * rwmi.h -- C ABI of the MI355X (gfx950) library for one coupled time step of
 * the random-walk / metaball / lattice-Boltzmann method of arXiv 2308.05007
 * ("RW-MI-DELBM").
 *
 * The library advances, entirely in hand-written HIP kernels:
 *   - a D3Q19 BGK lattice Boltzmann fluid (Sec. 2.3, Eq. 12-15) coupled to
 *     moving metaball particles (Eq. 3) through partially saturated cells
 *     (named in Sec. 1), with Guo body forcing and halfway bounce-back walls
 *     carrying the moving-wall term of Eq. 23;
 *   - N solute random walkers (Eq. 2): trilinear velocity interpolation
 *     (Sec. 2.4.1), Gaussian steps from Philox4x32-10, the four
 *     walker/particle types of Sec. 2.4.2 with Algorithm 1 (intersection by
 *     binary search), Algorithm 2 (specular reflection, Eq. 18-22) and the
 *     refill of swept walkers, reflection at walls.  The walker count is
 *     conserved exactly.
 *
 * Conventions shared by every call
 *   - Lattice units: dx = dt = 1.  Node (i,j,k) is centred at
 *     (i+1/2, j+1/2, k+1/2); its cell is [i,i+1) x [j,j+1) x [k,k+1).
 *     Linear node index = i + nx (j + ny k).  Arrays over nodes are SoA with x
 *     fastest.
 *   - D3Q19 direction order: rest; +x,-x,+y,-y,+z,-z; then (1,1,0),(-1,-1,0),
 *     (1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),(0,1,1),
 *     (0,-1,-1),(0,1,-1),(0,-1,1).  Weights 1/3, 1/18, 1/36; c_s^2 = 1/3.
 *   - A wall axis has solid wall nodes at index 0 and n-1; the halfway
 *     bounce-back planes sit at continuous coordinates 1 and n-1.
 *   - Every call returns an rwmi_status.  rwmi_last_error() gives a message
 *     owned by the library, valid until the next call on the same domain.
 *   - A domain is not thread-safe; distinct domains may be used from
 *     distinct threads.  Device work is enqueued on the domain's stream
 *     (the caller's hipStream_t, or one the library creates); calls named
 *     read_* synchronise that stream, rwmi_step does not.
 *   - Host pointers passed in are read during the call only; the caller keeps
 *     ownership.  Host output buffers are caller-allocated with the sizes
 *     from rwmi_query_sizes().
 */
#ifndef RWMI_H
#define RWMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RWMI_OK = 0,
  RWMI_EINVAL = -1,  /* an argument is out of range; nothing was changed */
  RWMI_ENOMEM = -2,  /* device allocation failed */
  RWMI_EDEVICE = -3, /* a HIP call failed (message in rwmi_last_error) */
  RWMI_ESTATE = -4,  /* call not allowed in the current state */
  RWMI_ESEED = -5    /* a walker found no admissible position */
} rwmi_status;

typedef enum { RWMI_BC_PERIODIC = 0, RWMI_BC_WALL = 1 } rwmi_bc;

/* Storage/compute modes.  FP64: distributions, velocity and walker offsets in
 * double, arithmetic in double with no contraction (reproduces the FP64
 * reference bit for bit).  FP32 / FP16_STORE / BF16_STORE: distributions
 * stored as deviations f_i - w_i rho0 in float / half / bfloat16, collision
 * in float, velocity field in float, walker offsets in float.  Every mode
 * draws its Gaussian normals from the same Philox words (FP64 with an exact
 * double Box-Muller, the others with the float hardware log / sin / cos), so
 * the walkers of all modes see the same noise up to float rounding. */
typedef enum { RWMI_FP64 = 0, RWMI_FP32 = 1, RWMI_FP16_STORE = 2, RWMI_BF16_STORE = 3 } rwmi_precision;

/* Motion of a particle.  Prescribed rigid motion (fixed orientation; the
 * oscillator of Sec. 4 read as a displacement sinusoid):
 *   STATIC   c(t) = c0
 *   SINUSOID c(t) = c0 + A sin(2 pi (t / period + phase)),  phase in cycles
 *   CONST_VEL c(t) = c0 + v t
 * The surface velocity seen by the fluid is dc/dt (Sec. 2.4.3 with w = 0).
 *   COUPLED  Newton-Euler motion (Sec. 2.2, Eq. 4) under gravity, the drive
 *            of Eq. 37, the hydrodynamic force and torque and the contacts
 *            of Eq. 5-11 (rwmi_set_coupling); surface velocity v + w x r;
 *            the initial velocity is the descriptor's `velocity`. */
typedef enum {
  RWMI_MOTION_STATIC = 0,
  RWMI_MOTION_SINUSOID = 1,
  RWMI_MOTION_CONST_VEL = 2,
  RWMI_MOTION_COUPLED = 3
} rwmi_motion;

/* Walker release (Sec. 3.1 point source, Sec. 4 solute band):
 *   UNIFORM  uniform over the fluid box
 *   GAUSSIAN centre + sigma z, z standard normal
 *   BAND     uniform, except axis band_axis uniform in [band_lo, band_hi)
 *   EXPLICIT the host positions xyz (3 per walker, continuous coordinates) */
typedef enum { RWMI_SEED_UNIFORM = 0, RWMI_SEED_GAUSSIAN = 1, RWMI_SEED_BAND = 2, RWMI_SEED_EXPLICIT = 3 } rwmi_seed_kind;

typedef void* (*rwmi_alloc_fn)(size_t bytes, void* ctx);
typedef void (*rwmi_free_fn)(void* ptr, void* ctx);

typedef struct {
  int32_t n[3];             /* lattice nodes per axis (>= 1; >= 3 on a wall axis) */
  int32_t bc[3];            /* rwmi_bc per axis */
  double wall_u_lo[3][3];   /* [axis][component] velocity of the wall at index 0 */
  double wall_u_hi[3][3];   /* [axis][component] velocity of the wall at index n-1 */
  double tau;               /* BGK relaxation time, > 0.5 (Eq. 12) */
  double force[3];          /* uniform body force per unit volume (Guo forcing) */
  double diffusivity;       /* solute D >= 0 (Eq. 1-2) */
  double rho0;              /* initial density (0 means 1) */
  double u0[3];             /* initial uniform velocity */
  uint64_t seed;            /* Philox key = (seed mod 2^32, seed >> 32) */
  int32_t precision;        /* rwmi_precision */
  int32_t device;           /* HIP device ordinal */
  void* stream;             /* hipStream_t to enqueue on, or NULL for a library stream */
  rwmi_alloc_fn alloc;      /* optional device allocator (e.g. the torch caching */
  rwmi_free_fn free;        /*   allocator); NULL pair means hipMalloc / hipFree  */
  void* alloc_ctx;
} rwmi_domain_desc;

typedef struct {
  int32_t n_ctrl;           /* control points, 1..RWMI_MAX_CTRL */
  const double* offsets;    /* 3*n_ctrl: control point - centre, world frame (Eq. 3 x_i) */
  const double* weights;    /* n_ctrl: k_i > 0 (Eq. 3) */
  double centre[3];         /* c0 */
  int32_t motion;           /* rwmi_motion */
  double amplitude[3];      /* SINUSOID amplitude vector A */
  double period;            /* SINUSOID period in steps (> 0) */
  double phase;             /* SINUSOID phase in cycles */
  double velocity[3];       /* CONST_VEL velocity */
} rwmi_metaball_desc;

typedef struct {
  int32_t kind;             /* rwmi_seed_kind */
  double centre[3];         /* GAUSSIAN centre */
  double sigma;             /* GAUSSIAN standard deviation */
  int32_t band_axis;        /* BAND axis (0..2) */
  double band_lo, band_hi;  /* BAND range along that axis */
  const double* xyz;        /* EXPLICIT positions, 3 per walker (host) */
  double ref[3];            /* reference point for the position moments */
  int32_t max_attempts;     /* redraws per walker (0 means 64) */
  int32_t remove_inside;    /* 1: drop (not redraw) walkers inside a particle, the
                               paper's removal at the first step (Sec. 2.4.2) */
} rwmi_seed_desc;

/* FP64 moments of the state after the last completed step (Eq. 16, Eq. 38-40
 * inputs).  Walker positions are unwrapped with their periodic image counts;
 * sums run over walkers, field sums over fluid (non-wall) nodes, with eps the
 * solid fraction of the last fluid update. */
typedef struct {
  uint64_t step;            /* completed coupled steps */
  uint64_t n_walkers;       /* exact walker count */
  double sum[3];            /* sum (X - ref) */
  double sumsq[3];          /* sum (X - ref)^2 */
  double mass;              /* sum rho */
  double momentum[3];       /* sum rho u */
  double fluid_u[3];        /* sum (1-eps) u / sum (1-eps) */
  double particle_v[3];     /* sum eps u_s / sum eps (0 without solid) */
  double solid_volume;      /* sum eps */
  uint64_t type2;           /* walkers inside a particle at both ends (refilled) */
  uint64_t type4;           /* walkers entering a particle (reflected, Alg. 1-2) */
  uint64_t bisect_fail;     /* Algorithm 1 reached its iteration cap */
  uint64_t refill_fallback; /* refill found no admissible point */
  uint64_t returned_to_origin; /* narrow-gap rule: walker kept its position */
  uint64_t wall_reflect;    /* walkers reflected at a wall */
  uint64_t near_surface;    /* walker steps that took the near-surface path (a cost
                               diagnostic: it depends on the culling, not a result) */
  uint64_t contact_misses;  /* coupled-particle steps that moved farther than half the
                               contact candidate margin (contacts may have been missed;
                               0 in any run within the model's speed limits) */
} rwmi_moments;

/* Two-way coupling of the particles with motion COUPLED (Sec. 2.2, Eq. 4-11;
 * the hydrodynamic force of the partially saturated cells).  Lattice units
 * (fluid density rho0 = 1, one fluid step = unit time). */
typedef struct {
  double density;            /* particle density rho_p > 0 */
  double gravity[3];         /* g of Eq. 4 */
  double drive_amplitude;    /* Eq. 37: acceleration a cos(2 pi t / T) along d */
  double drive_period;       /*   T in steps (> 0) */
  double drive_direction[3]; /*   d (unit vector) */
  double kn, kt;             /* Eq. 5: normal (> 0) and tangential (>= 0) stiffness */
  double eta_n, eta_t;       /*   normal and tangential damping (>= 0) */
  double mu;                 /*   friction coefficient (>= 0) */
  double dilation_radius;    /* R_s of the sphero-metaball contact (Eq. 9, 11) */
  int32_t substeps;          /* particle substeps per fluid step (1..1024) */
  int32_t coupling;          /* 1: the fluid's force and torque act on the particles */
} rwmi_coupling_desc;

typedef struct rwmi_domain rwmi_domain;
typedef struct rwmi_batch rwmi_batch;

#define RWMI_MAX_PARTICLES 64
#define RWMI_MAX_CTRL 64

/* Create a domain: allocates the lattice state on the device and sets every
 * distribution to the equilibrium of (rho0, u0) (Eq. 13).  *out owns the
 * device memory until rwmi_destroy_domain.  EINVAL on bad sizes, tau <= 0.5,
 * D < 0, unknown precision; ENOMEM / EDEVICE on device failure. */
rwmi_status rwmi_create_domain(const rwmi_domain_desc* desc, rwmi_domain** out);

/* Release every device buffer of the domain (after synchronising its stream).
 * NULL is ignored.  A domain still in a batch is removed from it first. */
void rwmi_destroy_domain(rwmi_domain* dom);

/* Add a metaball particle (Eq. 3) with prescribed motion.  The host arrays are
 * copied.  *out_id receives its index (0-based, in call order; lower indices
 * win where particles overlap).  ESTATE once walkers are seeded or a step has
 * run; EINVAL on n_ctrl out of range, a weight <= 0, period <= 0, or more
 * than RWMI_MAX_PARTICLES particles. */
rwmi_status rwmi_add_metaball_particle(rwmi_domain* dom, const rwmi_metaball_desc* p, int32_t* out_id);

/* Set up the two-way coupling of the particles added with motion COUPLED
 * (Sec. 2.2, Eq. 4-11); call after adding the particles and before seeding
 * and stepping.  For each such particle: the mass, centre of mass and
 * inertia tensor of the body M >= 1 at density rho_p (cells of size rb/24
 * weighted by their solid fractions); the centre of mass becomes the
 * particle's centre (the body stays where it was given), orientation the
 * identity, angular momentum zero.  Contacts act between coupled particles
 * and between them and the wall planes (1 and n - 1 on a wall axis); the
 * inner body is the level set M = (sqrt K / (sqrt K - R_s))^2, K = sum k_i.
 * Each step then runs the fluid at P(t), which sums the momentum its solid
 * term takes from the fluid, -sum_i e_i B Om_i per node, shared among the
 * coupled particles covering the node in proportion to their solid fractions
 * (fixed point, 2^-48: independent of the summation order); then the
 * particle update to t+1 in `substeps` symplectic Euler substeps with that
 * force and torque held constant; then the walkers against P(t+1).  The
 * domain steps with 256 threads per block, three launches per step, and
 * cannot join a batch.  EINVAL: no coupled particle, parameters out of
 * range, a particle with sqrt K <= R_s, more than 1024 control points in
 * all; ESTATE: after seeding, stepping or a second call. */
rwmi_status rwmi_set_coupling(rwmi_domain* dom, const rwmi_coupling_desc* c);

/* Fluid-particle coupling of a domain (Sec. 2.4.3):
 *   PSM  partially saturated cells (the default): the solid fraction of each
 *        node (Eq. 3, Eq. 17) weights a Noble-Torczynski solid term in the
 *        collision;
 *   IBB  interpolated bounce-back, the paper's own rule (Eq. 23-27): a node
 *        whose centre is inside a particle is solid (no collision, its
 *        velocity the particle's v + w x r); a fluid node whose upstream
 *        neighbour along e_i was solid at the previous update receives
 *        Eq. 23 with Eq. 24 (equilibrium at u_d plus its own post-collision
 *        non-equilibrium part) and Eq. 25 for u_d, q the fraction of the
 *        link to the surface M = 1 (a bracketed regula falsi); a node uncovered since the
 *        previous update restarts from f^eq(rho0, u_new) (Eq. 27); the
 *        force on coupled particles is the links' Galilean-invariant
 *        momentum exchange, applied in the particle update of the next
 *        step. */
typedef enum { RWMI_COUPLING_PSM = 0, RWMI_COUPLING_IBB = 1 } rwmi_coupling;

/* Choose the fluid-particle coupling (rwmi_coupling) before the first step.
 * IBB switches the domain to two lattices and 256 threads per block, and
 * keeps one status byte per node per step parity; such a domain cannot join
 * a batch.  EINVAL for an unknown scheme; ESTATE after stepping or inside a
 * batch. */
rwmi_status rwmi_set_fluid_coupling(rwmi_domain* dom, int32_t scheme);

/* State of coupled particle p after the last completed step, 32 doubles:
 * centre of mass c[3], velocity v[3], orientation quaternion q[4] (w, x, y,
 * z; body to world), angular momentum L[3], angular velocity w[3], the
 * hydrodynamic force F_h[3] and torque T_h[3] of the last fluid step, mass,
 * body-frame inertia tensor I[9] (row-major).  Synchronises the domain's
 * stream.  EINVAL if p is not a coupled particle. */
rwmi_status rwmi_read_particle_state(rwmi_domain* dom, int32_t p, double* out);

/* Replace the velocity and angular momentum of coupled particle p (host
 * arrays of 3) at the current step; the angular velocity follows as
 * R I_b^-1 R^T L.  Synchronises the domain's stream.  EINVAL if p is not a
 * coupled particle. */
rwmi_status rwmi_set_particle_motion(rwmi_domain* dom, int32_t p, const double v[3], const double L[3]);

/* Seed n walkers (ids 0..n-1) at step 0, on the device: the solute particles
 * of the random-walk method (Sec. 2.4, Eq. 2), released as in the paper's
 * tests (a point or a Gaussian pulse, Sec. 3.1; a horizontal band, Sec. 4)
 * or uniformly in the fluid; the concentration they carry is the node count
 * of Eq. 16.  Attempt a of walker
 * w draws the Philox block with counter (w, 0xFFFFFFFF, 16 + a, 0); positions
 * inside a particle at t = 0 or outside the fluid range of a wall axis are
 * redrawn up to max_attempts times (remove_inside = 1: dropped instead, the
 * survivors keep their order and are renumbered).  *out_seeded receives the
 * number placed.  ESEED if a walker ran out of attempts (the placed walkers
 * are kept); ESTATE after the first step or a second call; EINVAL for a bad
 * kind or n > 2^31 - 1. */
rwmi_status rwmi_seed_walkers(rwmi_domain* dom, const rwmi_seed_desc* s, uint64_t n, uint64_t* out_seeded);

/* Enqueue n_steps coupled steps t -> t+1 on the domain's stream and return.
 * Each step (the coupled scheme of Sec. 2.4 on the lattice Boltzmann update
 * of Sec. 2.3, Eq. 12-15, and the random-walk update of Eq. 2): particle
 * poses at t and t+1 (prescribed motion, Sec. 4 Eq. 37); fluid update at P(t)
 * writing u(t); walkers moved with u(t) (Sec. 2.4.1) and classified against
 * P(t+1) (types I-IV, Sec. 2.4.2; Algorithms 1-2); walker counter
 * (w, t, purpose, 0) with purpose 0 Brownian, 1 refill direction, 2 refill
 * radius.  n steps are n + 1 launches of one fused kernel on the domain
 * stream (launch j: fluid and prologue of step t0 + j, walkers of step
 * t0 + j - 1).  Device-side anomalies are counted (see rwmi_moments), never
 * returned. */
rwmi_status rwmi_step(rwmi_domain* dom, uint32_t n_steps);

/* Compute and copy the FP64 moments (synchronises). */
rwmi_status rwmi_read_moments(rwmi_domain* dom, rwmi_moments* out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same moments,
 * bit for bit, from the same kernels, with no allocation of any kind.  The
 * reduction's partials, staging output and reference point live in one
 * file-scope device array of the library, 1 MiB per GPU (131072 doubles),
 * which each GPU the library runs on holds until the process ends.  Limit:
 * 64 + 6 ceil(n_walkers / 4096) + 12 ceil(n_nodes / 4096) <= 131072 (the
 * 256^3 lattice with 1e7 walkers uses 49%); EINVAL beyond it, with the sizes
 * in the message.  ESTATE if the domain has particles and has been neither
 * seeded nor stepped (their upload allocates).  Synchronises the domain's
 * stream.  Every call on a GPU shares that GPU's array: calls for domains of
 * one GPU that overlap in time (from several host threads) race and must be
 * serialised by the caller. */
rwmi_status rwmi_read_moments_noalloc(rwmi_domain* dom, rwmi_moments* out);

/* Occupancy n_s per node (Eq. 16: walkers whose cell is the node), exact
 * uint32, nx*ny*nz entries (synchronises). */
rwmi_status rwmi_read_occupancy(rwmi_domain* dom, uint32_t* ns);

/* Concentration profile along an axis: counts[k] = the number of walkers
 * whose cell lies in layer k of that axis (Eq. 16 summed over the two other
 * axes; Sec. 4 averages such profiles over realisations and fits a Gaussian
 * to them).  n[axis] entries, exact; synchronises.  EINVAL for an axis
 * outside 0..2. */
rwmi_status rwmi_read_profile(rwmi_domain* dom, int32_t axis, uint64_t* counts);

/* Velocity u(t) of the last fluid update, SoA [3][nodes] as double, and the
 * density of that update (rho may be NULL).  Wall nodes carry the wall
 * velocity.  Before any step: u0 and rho0. */
rwmi_status rwmi_read_velocity(rwmi_domain* dom, double* u, double* rho);

/* Walker state: cell index (int32, n entries), offsets in [0,1) SoA [3][n]
 * as double, periodic image counts SoA [3][n] (any pointer may be NULL). */
rwmi_status rwmi_read_walkers(rwmi_domain* dom, int32_t* cell, double* off, int32_t* img);

/* Pre-collision distributions f_i(x, t) at the current step, SoA [19][nodes]
 * as double (wall nodes: unspecified).  Diagnostic. */
rwmi_status rwmi_read_distributions(rwmi_domain* dom, double* f);

/* Sizes for the read buffers and the number of steps enqueued so far. */
rwmi_status rwmi_query_sizes(const rwmi_domain* dom, uint64_t* n_nodes, uint64_t* n_walkers, uint64_t* step);

/* Device bytes a domain with these parameters holds (for admission by HBM
 * footprint).  Does not touch the device. */
uint64_t rwmi_footprint_bytes(const rwmi_domain_desc* desc, uint32_t n_particles, uint32_t n_ctrl_total,
                              uint64_t n_walkers);

/* Debug and tuning knobs (EINVAL on an unknown key):
 *   RWMI_KEY_MAX_BISECT      iteration cap of Algorithm 1 (default 200, >= 1)
 *   RWMI_KEY_USE_GRAPH       0/1: replay steps from a captured hipGraph
 *   RWMI_KEY_BLOCK           threads per block of the step launch (128, 256, 512;
 *                            default 256): nodes per fluid block, walkers per
 *                            walker block, mask blocks per prologue block
 *   RWMI_KEY_TIMING          p > 0: record HIP events around windows of p consecutive
 *                            step launches (1: every launch on its own); 0: off
 *   RWMI_KEY_STEP_FLAGS      launch options of the step kernel: bit 0 deals each of
 *                            the 8 XCDs a contiguous run of fluid blocks with its
 *                            share of walker blocks interleaved (default on), bit 1
 *                            writes f* and u with non-temporal stores
 *   RWMI_KEY_SORT_EVERY      regroup the walkers by coarse block (4^3 nodes) every this
 *                            many steps for memory locality (default 128, 0 = never)
 *   RWMI_KEY_STREAMING       1: two lattices (pull from one, write the other); 2: one
 *                            lattice streamed in place.  Default: in place while the 19
 *                            distributions take at most 384 MB, else two lattices.
 *                            Only before the first step (ESTATE after); resets f to f^eq
 * Results never depend on the block size, flags or sort interval: walker ids
 * travel with the walkers and every read-out is by id. */
enum {
  RWMI_KEY_MAX_BISECT = 1,
  RWMI_KEY_USE_GRAPH = 2,
  RWMI_KEY_BLOCK = 3,
  RWMI_KEY_TIMING = 5,
  RWMI_KEY_STEP_FLAGS = 6,
  RWMI_KEY_SORT_EVERY = 7,
  RWMI_KEY_STREAMING = 8,
  RWMI_KEY_MEMBER_BLOCKS = 10
};
rwmi_status rwmi_debug_set(rwmi_domain* dom, int32_t key, int64_t value);

/* Timing of the step launches recorded while RWMI_KEY_TIMING is on
 * (synchronises, then clears the record): *ms total milliseconds between the
 * events bracketing each timed window of consecutive step launches (windows
 * close before a walker regrouping and at the end of a launch group, so they
 * hold step launches only), *launches the launches timed, and how many of
 * them carried a fluid update (*fluid_steps) and a walker step
 * (*walker_steps); a group of n steps is n + 1 launches, the first without
 * walkers, the last with walkers only. */
rwmi_status rwmi_read_kernel_times(rwmi_domain* dom, double* ms, uint64_t* launches, uint64_t* fluid_steps,
                                   uint64_t* walker_steps);

/* With coupled particles (rwmi_set_coupling) and RWMI_KEY_TIMING on, each
 * launch of a step is timed on its own: the step launches go to the record
 * above (one launch per window), the particle updates and the prologues
 * that build the masks at the new poses to this one.  Synchronises, returns
 * their total milliseconds and counts, then clears this record. */
rwmi_status rwmi_read_coupling_times(rwmi_domain* dom, double* ms_update, uint64_t* n_update, double* ms_prologue,
                                     uint64_t* n_prologue);

/* Block until all work enqueued for the domain has finished. */
rwmi_status rwmi_synchronize(rwmi_domain* dom);

/* Message of the last failing call on dom (dom NULL: of the last failing
 * create / batch call on this thread).  Never NULL. */
const char* rwmi_last_error(const rwmi_domain* dom);

/* ---------------------------------------------------------------- batch
 * A batch steps many domains with one fused launch per step and precision
 * (block maps over all member domains) on the batch stream, optionally replayed
 * from a hipGraph.  Members keep their state and ownership; results of a
 * domain are bit-identical to stepping it alone (same arithmetic per node and
 * per walker).  Members must live on the batch device; their own streams are
 * synchronised before each batch step.  rwmi_batch_add returns EINVAL for a
 * domain with two-way coupled particles (rwmi_set_coupling) or with the
 * bounce-back coupling (rwmi_set_fluid_coupling): such domains step alone,
 * and ESTATE for a domain already in a batch. */
rwmi_status rwmi_batch_create(int32_t device, void* stream, rwmi_batch** out);
rwmi_status rwmi_batch_add(rwmi_batch* b, rwmi_domain* dom);
rwmi_status rwmi_batch_remove(rwmi_batch* b, rwmi_domain* dom);
/* Enqueue n_steps steps of every member on the batch stream. */
rwmi_status rwmi_batch_step(rwmi_batch* b, uint32_t n_steps);
/* Launch options of the batch (RWMI_KEY_USE_GRAPH, _BLOCK, _STEP_FLAGS); they
 * replace the members' own for batch steps.  RWMI_KEY_MEMBER_BLOCKS = 1: each
 * member launches with its own block size (RWMI_KEY_BLOCK of that domain, which
 * may be set while it is in the batch), so that every size class of a mixed
 * batch has its own launch shape; the members of one precision, layout and
 * block size share each launch, and all launches of a step are captured in
 * one graph.  0 (default): every member uses the batch's RWMI_KEY_BLOCK. */
rwmi_status rwmi_batch_set(rwmi_batch* b, int32_t key, int64_t value);
rwmi_status rwmi_batch_synchronize(rwmi_batch* b);
void rwmi_batch_destroy(rwmi_batch* b);

/* ---------------------------------------------------------------- dispersion
 * Dispersion coefficient from a series of solute moments (Sec. 4, Eq. 38-40):
 * with s_i = sigma2[i] / two_r^2 the least-squares line s = a + b t over the
 * samples i0..n-1 gives the slope b = K u_slip / two_r of Eq. 38, so
 * K = b two_r / u_slip, and D_alpha = K / (1 - phi) (Eq. 40).  sigma2[i] is
 * the variance of the walker positions along the dispersion axis at time
 * t[i] (sumsq/N - (sum/N)^2 of rwmi_moments); u_slip = <u> - <u_p> (Eq. 39);
 * phi the solid volume fraction.  Host-only arithmetic on caller arrays.
 * EINVAL if fewer than 2 samples are used, u_slip == 0 or phi >= 1. */
rwmi_status rwmi_dispersion_fit(const double* t, const double* sigma2, uint32_t n, uint32_t i0, double two_r,
                                double u_slip, double phi, double* K, double* D_alpha, double* offset);

/* The dispersion pipeline of Sec. 4 (Eq. 38-40) from a series of moment
 * read-outs of one domain (rwmi_read_moments every m steps), host-only
 * arithmetic on the caller's array:
 *   sigma2_i = sumsq[a]/N_w - (sum[a]/N_w)^2 of sample i along the dispersion
 *              axis a (the variance of the unwrapped walker positions; the
 *              Gaussian-fit variance of the averaged concentration profile);
 *   u_slip   = |max_i fluid_u[f] - max_i particle_v[f]| along the flow axis f
 *              (Eq. 39: the maxima over time of the fluid-average and the
 *              particle-average velocity; the magnitude, since with
 *              prescribed particle motion the fluid lags the particles);
 *   phi      = mean of solid_volume over the samples taken after at least
 *              one step, divided by n_nodes (the solid volume fraction);
 *   K, D_alpha, offset from rwmi_dispersion_fit on (step_i, sigma2_i),
 *              i = i0..n-1, with two_r the particle diameter (Eq. 38, 40).
 * sigma2 (n doubles) receives the variance series if not NULL.  EINVAL if
 * fewer than 2 samples are fitted, a sample has no walkers, an axis is not
 * 0..2, n_nodes is 0, u_slip is 0 or phi >= 1. */
typedef struct {
  double u_slip;
  double phi;
  double K;
  double D_alpha;
  double offset;
} rwmi_dispersion;
rwmi_status rwmi_dispersion_from_moments(const rwmi_moments* series, uint32_t n, uint32_t i0, int32_t disp_axis,
                                         int32_t flow_axis, uint64_t n_nodes, double two_r, double* sigma2,
                                         rwmi_dispersion* out);

/* Least-squares Gaussian y = amp exp(-(x - mean)^2 / (2 var)) through n
 * points (Sec. 4: Gaussian distributions fitted to the averaged
 * concentration profiles give the variance series of Eq. 38), by
 * Levenberg-Marquardt from the profile's weighted moments.  Host-only
 * arithmetic on caller arrays.  EINVAL if fewer than three y are positive
 * (three parameters are not fixed by fewer points). */
rwmi_status rwmi_gaussian_fit(const double* x, const double* y, uint32_t n, double* amp, double* mean, double* var);

/* ---------------------------------------------------------------- diagnostics
 * The Gaussian triples the walker kernels draw for counters (id, t, purpose,
 * 0), id = 0..n-1, under key seed, written as n x 3 doubles to host z. */
rwmi_status rwmi_device_normals(int32_t device, uint64_t seed, uint32_t t, uint32_t purpose, uint64_t n, double* z);

/* Bandwidth probe of the lattice update's memory pattern without its
 * arithmetic or neighbour shifts: one launch on `stream` (a hipStream_t;
 * NULL: the null stream) in which each of n nodes reads one element from
 * each of `streams` arrays of src and writes one to each of as many arrays
 * of dst, 2 * elem_bytes * streams * n bytes in all.  Elements are floats
 * (elem_bytes 4) or IEEE halves (2, the 16-bit storage modes).  tiled = 0:
 * array i of node k at i * n + k; tiled = 1: in tiles of 256 nodes, the
 * tile's 256 values of array 0, then of array 1, and so on (the
 * distributions' two-lattice layout).  src and dst are device buffers of
 * streams * n elements owned by the caller.  Asynchronous: returns after
 * the launch.  EINVAL unless streams is 1, 2, 4, 8 or 19, elem_bytes is 4
 * or 2, n is a positive multiple of 256 below 2^32 and both pointers are
 * non-NULL; EDEVICE if the launch fails. */
rwmi_status rwmi_stream_probe(int32_t streams, int32_t elem_bytes, int32_t tiled, uint64_t n, const void* src,
                              void* dst, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RWMI_H */
