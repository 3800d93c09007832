// The fused step launch: walker blocks of step t-1, fluid blocks of step t
// and prologue blocks of step t+1 in one grid (roles from step_map.h), t being
// the domain's step counter at the start of the launch group plus the launch
// index j.  A group of n steps is a prologue-only launch (j = -1, prologue of
// t0) and then launches j = 0..n: fluid of t0 + j (j < n), prologue of
// t0 + j + 1 (j < n - 1), walkers of t0 + j - 1 (j >= 1).
//
// No role reads what another role of the same launch writes.  The fluid of
// step t reads f of parity t & 1, the poses of slot t mod 3 and writes f, u of
// parity (t + 1) & 1 and t & 1 (and, on the group's last fluid step, the
// densities, which no role reads); the walkers of step t - 1 read u of parity
// (t - 1) & 1 and the poses/mask of slot (t - 1) mod 3; the prologue writes
// slot (t + 1) mod 3.
#pragma once
#include "lbm_impl.h"
#include "pro_impl.h"
#include "step_map.h"
#include "walk_impl.h"

namespace rwmi {

template <int P, int BS>
union StepLds {
  WalkLds<typename Store<P>::O, BS> walk;
  ProLds pro;
  unsigned long long dem[6 * kMaxParticles];  // fluid blocks with coupled particles
};

// IP: the domains of the launch stream their lattice in place (else: two
// lattices); one instantiation per layout keeps each kernel's registers to
// the paths it can take.
#ifndef RWMI_STEP_WAVES_PER_EU_32
#define RWMI_STEP_WAVES_PER_EU_32 6
#endif
#ifndef RWMI_STEP_WAVES_PER_EU_16
#define RWMI_STEP_WAVES_PER_EU_16 8
#endif
// Waves per SIMD the register allocation must leave room for, measured on
// the 256^3 oscillator.  FP32 storage: 6 (69 VGPRs, 7 waves, no spill) runs
// the step in 609 us against 621 us at 8 (63 VGPRs and a few spills to
// scratch); 16-bit storage the other way round, 413 us at 8 against 431 us
// at 6.  FP64 needs about twice the registers: no constraint.
template <int P, bool IBB = false>
constexpr int step_waves_per_eu() {
  return P == P64 ? 1 : (P == P32 ? RWMI_STEP_WAVES_PER_EU_32 : RWMI_STEP_WAVES_PER_EU_16);
}

// DEM: the launch's domains have two-way coupled particles (the fluid
// blocks accumulate the hydrodynamic force and torque on them).  IBB: they
// couple fluid and particles by interpolated bounce-back (two lattices).
template <int P, int BS, bool IP, bool DEM = false, bool IBB = false>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(step_waves_per_eu<P, IBB>())))
k_step(StepArgs a, const DomView* __restrict__ views, const int32_t* __restrict__ boff) {
  // views and boff (the same pointers as in a) are read-only in the launch:
  // as restrict parameters their wave-uniform reads compile to scalar loads
  __shared__ StepLds<P, BS> lds;
  int idx = 0;
  const int role = step_role((int)blockIdx.x, a.nb, (a.flags & 1) != 0, idx);
  if (role == kRoleNone) return;
  const int32_t* bo = boff + role * (a.nd + 1);
  const int d = find_domain(bo, a.nd, idx);
  const DomView& V = views[d];
  const int lb = idx - bo[d];
  const uint64_t t = step_of(V, a.j);
  if (role == kRoleWalk) walk_block<P, BS>(V, lb, t - 1, lds.walk);
  else if (role == kRolePro) prologue_block(V, lb, t + 1, BS, lds.pro, (a.flags & kFlagDem) != 0);
  else {
    const bool nt = (a.flags & kFlagNontemporal) != 0, dens = (a.flags & kFlagDensity) != 0;
    if constexpr (!IP) fluid_block<P, BS, kTwoLattices, DEM, IBB>(V, (uint32_t)lb, t, nt, dens, lds.dem);
    else if (t & 1ull) fluid_block<P, BS, kInPlaceOdd, DEM>(V, (uint32_t)lb, t, nt, dens, lds.dem);
    else fluid_block<P, BS, kInPlaceEven, DEM>(V, (uint32_t)lb, t, nt, dens, lds.dem);
  }
}

}  // namespace rwmi
