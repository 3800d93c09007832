/* A plain C client of the rwmi C ABI (include/rwmi.h): no Python and no
 * PyTorch.  The library allocates the device memory (hipMalloc) and creates
 * the stream itself.  It builds one FP64 domain, adds a metaball particle on
 * a sinusoidal path, seeds uniform walkers, steps, and prints the moments of
 * the final state one value per line: doubles as exact hexadecimal floats,
 * counters as decimal integers.  A velocity read-out and the cell occupancy
 * are printed as their sums.
 *
 *   abi_client STEPS COUPLING     COUPLING 0: partially saturated cells,
 *                                 1: interpolated bounce-back (Eq. 23-27)
 *
 * Exit status 0 on success; on an error it prints the library's message to
 * stderr and returns 1. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rwmi.h"

static int bad(rwmi_status st, const rwmi_domain* d, const char* what) {
  if (st == RWMI_OK) return 0;
  fprintf(stderr, "%s failed (%d): %s\n", what, (int)st, rwmi_last_error(d));
  return 1;
}

int main(int argc, char** argv) {
  const int steps = argc > 1 ? atoi(argv[1]) : 40;
  const int coupling = argc > 2 ? atoi(argv[2]) : 0;

  rwmi_domain_desc dd;
  memset(&dd, 0, sizeof dd);
  const int32_t n[3] = {20, 14, 24};
  for (int a = 0; a < 3; ++a) {
    dd.n[a] = n[a];
    dd.bc[a] = a == 1 ? RWMI_BC_WALL : RWMI_BC_PERIODIC;
  }
  dd.wall_u_hi[1][0] = 0.01; /* the upper y wall slides along x */
  dd.tau = 0.8;
  dd.force[0] = 1e-5;
  dd.diffusivity = 0.02;
  dd.rho0 = 1.0;
  dd.seed = 0x1234567890abcdefull;
  dd.precision = RWMI_FP64;
  dd.device = 0;
  dd.stream = NULL;
  rwmi_domain* d = NULL;
  if (bad(rwmi_create_domain(&dd, &d), NULL, "rwmi_create_domain")) return 1;

  const double offsets[6] = {-0.8, 0.0, 0.0, 0.8, 0.3, 0.0};
  const double weights[2] = {0.6, 0.5};
  rwmi_metaball_desc mb;
  memset(&mb, 0, sizeof mb);
  mb.n_ctrl = 2;
  mb.offsets = offsets;
  mb.weights = weights;
  mb.centre[0] = 10.0;
  mb.centre[1] = 7.0;
  mb.centre[2] = 12.0;
  mb.motion = RWMI_MOTION_SINUSOID;
  mb.amplitude[0] = 1.5;
  mb.amplitude[2] = 0.5;
  mb.period = 30.0;
  mb.phase = 0.1;
  int32_t pid = -1;
  if (bad(rwmi_add_metaball_particle(d, &mb, &pid), d, "rwmi_add_metaball_particle")) return 1;
  if (coupling && bad(rwmi_set_fluid_coupling(d, RWMI_COUPLING_IBB), d, "rwmi_set_fluid_coupling")) return 1;

  rwmi_seed_desc sd;
  memset(&sd, 0, sizeof sd);
  sd.kind = RWMI_SEED_UNIFORM;
  sd.sigma = 1.0;
  sd.band_axis = 2;
  sd.band_lo = 0.0;
  sd.band_hi = 1.0;
  sd.ref[0] = 10.0;
  sd.ref[1] = 7.0;
  sd.ref[2] = 12.0;
  sd.max_attempts = 64;
  uint64_t seeded = 0;
  if (bad(rwmi_seed_walkers(d, &sd, 3000, &seeded), d, "rwmi_seed_walkers")) return 1;

  if (bad(rwmi_step(d, (uint32_t)steps), d, "rwmi_step")) return 1;
  if (bad(rwmi_synchronize(d), d, "rwmi_synchronize")) return 1;

  rwmi_moments m;
  if (bad(rwmi_read_moments(d, &m), d, "rwmi_read_moments")) return 1;
  const size_t N = (size_t)n[0] * n[1] * n[2];
  double* u = (double*)malloc(sizeof(double) * 3 * N);
  double* rho = (double*)malloc(sizeof(double) * N);
  uint32_t* occ = (uint32_t*)malloc(sizeof(uint32_t) * N);
  if (!u || !rho || !occ) return 1;
  if (bad(rwmi_read_velocity(d, u, rho), d, "rwmi_read_velocity")) return 1;
  if (bad(rwmi_read_occupancy(d, occ), d, "rwmi_read_occupancy")) return 1;
  double su[3] = {0.0, 0.0, 0.0};
  uint64_t socc = 0;
  for (size_t i = 0; i < N; ++i) {
    for (int a = 0; a < 3; ++a) su[a] += u[a * N + i];
    socc += occ[i];
  }

  printf("seeded %llu\n", (unsigned long long)seeded);
  printf("step %llu\n", (unsigned long long)m.step);
  printf("n_walkers %llu\n", (unsigned long long)m.n_walkers);
  for (int a = 0; a < 3; ++a) printf("sum%d %a\n", a, m.sum[a]);
  for (int a = 0; a < 3; ++a) printf("sumsq%d %a\n", a, m.sumsq[a]);
  printf("mass %a\n", m.mass);
  for (int a = 0; a < 3; ++a) printf("fluid_u%d %a\n", a, m.fluid_u[a]);
  printf("type2 %llu\n", (unsigned long long)m.type2);
  printf("type4 %llu\n", (unsigned long long)m.type4);
  printf("wall_reflect %llu\n", (unsigned long long)m.wall_reflect);
  printf("returned_to_origin %llu\n", (unsigned long long)m.returned_to_origin);
  for (int a = 0; a < 3; ++a) printf("usum%d %a\n", a, su[a]);
  printf("occupancy %llu\n", (unsigned long long)socc);
  free(u);
  free(rho);
  free(occ);
  rwmi_destroy_domain(d);
  return 0;
}
