// The fused step launch: walker blocks of step t-1, prologue blocks of step t
// and fluid blocks of step t in one grid (roles from step_map.h).  A launch
// group of n steps is n + 1 launches j = 0..n: launch j carries the fluid
// update and the prologue of step t0 + j (j < n) and the walkers of step
// t0 + j - 1 (j >= 1), t0 being the domain's step counter at the start of
// the group.  The walkers of step t read u(t) and the poses/mask of step t,
// written by the previous launch into the buffers of parity t & 1, while the
// current launch writes those of parity (t + 1) & 1.
#pragma once
#include "lbm_impl.h"
#include "pro_impl.h"
#include "step_map.h"
#include "walk_impl.h"

namespace rwmi {

template <int P, int BS>
union StepLds {
  BlockParticles fluid;
  WalkLds<typename Store<P>::O, BS> walk;
  ProLds pro;
};

template <int P, int BS>
__global__ void __launch_bounds__(BS) k_step(StepArgs a) {
  __shared__ StepLds<P, BS> lds;
  int idx = 0;
  const int role = step_role((int)blockIdx.x, a.nb, (a.flags & 1) != 0, idx);
  if (role == kRoleNone) return;
  const int32_t* bo = a.boff + role * (a.nd + 1);
  const int d = find_domain(bo, a.nd, idx);
  const DomView& V = a.views[d];
  const int lb = idx - bo[d];
  const uint64_t t = step_of(V, a.j);
  if (role == kRoleWalk) walk_block<P, BS>(V, lb, t - 1, lds.walk);
  else if (role == kRolePro) prologue_block(V, lb, t, lds.pro);
  else fluid_block<P, BS>(V, (uint32_t)lb, t, (a.flags & 2) != 0, lds.fluid);
}

}  // namespace rwmi
