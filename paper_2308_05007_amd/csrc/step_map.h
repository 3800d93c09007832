// Block roles of the fused step launch (host and device).
//
// One launch of a step group carries three kinds of blocks: the walkers of
// step t-1 (fast path, then the block's own near-surface walkers), the fluid
// update of step t and the prologue of step t+1 (particle poses, coarse cull
// mask).  They read only what earlier launches wrote and write disjoint
// buffers (velocity double-buffered by step parity, pose table and mask by
// step mod 3), so they need no ordering among themselves.
//
// Hardware block i runs on XCD i mod 8.  With the XCD-aware map every XCD
// receives a contiguous run of the fluid blocks (neighbouring nodes share its
// L2), its share of the walker blocks interleaved evenly among them (latency-
// bound walker work overlaps bandwidth-bound fluid work on every CU), and its
// prologue blocks first.  Without it the roles are dealt the same way over the
// whole grid.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define RWMI_HD __host__ __device__
#else
#define RWMI_HD  // plain C++ (host-side tests)
#endif

namespace rwmi {

enum BlockRole { kRoleWalk = 0, kRolePro = 1, kRoleFluid = 2, kRoles = 3, kRoleNone = -1 };

constexpr int kFlagXcd = 1;          // XCD-aware role map
constexpr int kFlagNontemporal = 2;  // non-temporal stores of f* and u
// Set by the host (never by a caller) on the launch that carries the last
// fluid step of a launch group: that step also writes the node densities,
// which only read-outs use.
constexpr int kFlagDensity = 4;
// The domains have two-way coupled particles: the prologue builds the masks
// from the poses the particle update wrote (step_impl.h, pro_impl.h).
constexpr int kFlagDem = 8;
// The domains couple fluid and particles by interpolated bounce-back
// (lbm_impl.h); set by the host.
constexpr int kFlagIbb = 16;

struct DomView;

// One fused step launch over nd domains (kernel argument).
struct StepArgs {
  const DomView* views;
  const int32_t* boff;  // kRoles maps of nd + 1 block prefixes: walkers, prologue, fluid
  int nd;
  int nb[kRoles];       // blocks per role over all domains
  int flags;            // kFlagXcd | kFlagNontemporal | kFlagDensity
  int inplace;          // every domain of the launch streams its lattice in place
  int32_t j;            // launch index within the group (-1: the prologue-only launch)
};

// Share of XCD x of n items dealt in contiguous runs: count and first item.
RWMI_HD inline int xcd_count(int n, int x) { return (n >> 3) + (x < (n & 7) ? 1 : 0); }
RWMI_HD inline int xcd_first(int n, int x) { return x * (n >> 3) + (x < (n & 7) ? x : (n & 7)); }

// Grid size for nb[role] blocks per role.
RWMI_HD inline int step_grid(const int nb[3], bool xcd) {
  if (!xcd) return nb[0] + nb[1] + nb[2];
  int g = 0;
  for (int x = 0; x < 8; ++x) {
    const int t = xcd_count(nb[0], x) + xcd_count(nb[1], x) + xcd_count(nb[2], x);
    if (t > g) g = t;
  }
  return 8 * g;
}

// Role of hardware block i and its index among the blocks of that role
// (kRoleNone for the padding blocks of the XCD-aware grid).
RWMI_HD inline int step_role(int i, const int nb[3], bool xcd, int& idx) {
  int g = i, cw = nb[0], cp = nb[1], cf = nb[2], bw = 0, bp = 0, bf = 0;
  if (xcd) {
    const int x = i & 7;
    g = i >> 3;
    cw = xcd_count(nb[0], x);
    cp = xcd_count(nb[1], x);
    cf = xcd_count(nb[2], x);
    bw = xcd_first(nb[0], x);
    bp = xcd_first(nb[1], x);
    bf = xcd_first(nb[2], x);
  }
  if (g < cp) {
    idx = bp + g;
    return kRolePro;
  }
  const int h = g - cp, T = cw + cf;
  if (h >= T) return kRoleNone;
  // walker blocks spread evenly among the fluid blocks: position h is a
  // walker block when floor((h+1) cw / T) > floor(h cw / T)
  const int wa = (int)(((int64_t)h * cw) / T);
  const int wb = (int)(((int64_t)(h + 1) * cw) / T);
  if (wb > wa) {
    idx = bw + wa;
    return kRoleWalk;
  }
  idx = bf + (h - wa);
  return kRoleFluid;
}

}  // namespace rwmi
