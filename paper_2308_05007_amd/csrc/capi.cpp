// Host side of the rwmi C ABI (include/rwmi.h): domain and batch state,
// device memory, launch sequencing, graph capture, readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rwmi.h"
#include "dem_impl.h"
#include "dev_common.h"
#include "launch.h"

namespace rwmi {
// the bandwidth probe (probe.hip)
hipError_t launch_stream_probe(int streams, int elem, bool tiled, uint64_t n, const void* src, void* dst,
                               hipStream_t s);
}

using rwmi::DevParticle;
using rwmi::DomView;

namespace {

thread_local std::string g_err = "no error";

constexpr uint64_t kNeverSorted = ~0ull;  // sorted_at before the first regrouping
// Steps captured in one graph: the default regrouping interval, so that a
// replay (which regroups the walkers at its start) regroups no more often
// than eager stepping does.
constexpr uint32_t kGraphSteps = 128;

struct HostParticle {
  std::vector<double> b, k;
  double c0[3], amp[3], vel[3], period, phase;
  int motion;
};

struct Alloc {
  rwmi_alloc_fn fa = nullptr;
  rwmi_free_fn ff = nullptr;
  void* ctx = nullptr;
};

size_t elem_size(int prec) { return prec == RWMI_FP64 ? 8 : (prec == RWMI_FP32 ? 4 : 2); }

// One lattice streamed in place while the distributions take at most 384 MB:
// up to about that size the in-place pattern, partly served by the 256 MB
// memory-side cache, beats the two-lattice pull (measured with real data:
// 3-5% faster at 227-319 MB of distributions, 2-3% slower at 427-538 MB).
// Larger lattices keep two lattices.
constexpr uint64_t kInPlaceMaxBytes = 384ull << 20;
bool default_inplace(const rwmi_domain_desc& s) {
  const uint64_t N = (uint64_t)s.n[0] * s.n[1] * s.n[2];
  return 19 * N * elem_size(s.precision) <= kInPlaceMaxBytes;
}
size_t u_size(int prec) { return prec == RWMI_FP64 ? 8 : 4; }
size_t off_size(int prec) { return prec == RWMI_FP64 ? 8 : 4; }

using rwmi::kRoleFluid;
using rwmi::kRolePro;
using rwmi::kRoles;
using rwmi::kRoleWalk;

}  // namespace

struct rwmi_domain {
  rwmi_domain_desc desc{};
  int prec = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Alloc al;
  std::string err = "no error";
  std::vector<HostParticle> parts;
  std::vector<void*> owned;  // device allocations to release
  DomView hv{};
  DomView* dv = nullptr;    // device copy of hv
  int32_t* dboff = nullptr; // kRoles block maps of 2 entries each
  bool particles_uploaded = false;
  bool seeded = false;
  bool stepped = false;
  uint64_t steps = 0;
  double ref[3] = {0, 0, 0};
  int bs = 256;  // threads per block of the step launch
  int flags = rwmi::kFlagXcd;
  int sort_every = 128;    // regroup walkers by coarse block every this many steps (0: never)
  uint64_t sorted_at = kNeverSorted;  // step of the last regrouping (host view)
  rwmi::SortScratch sort{};
  bool use_graph = false;
  bool timing = false;
  uint32_t timing_every = 1;  // step launches per timed window
  hipGraphExec_t gexec = nullptr;
  uint32_t gsteps = 0;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  // A timed window: consecutive step launches bracketed by one event pair.
  struct TimedWindow {
    size_t ev;         // index of the start event (the stop event follows)
    uint32_t launches; // step launches in the window
    uint32_t fluid;    // of them, launches that carried a fluid update
    uint32_t walkers;  // and launches that carried a walker step
  };
  std::vector<TimedWindow> evrec;
  // coupled particles: timed particle updates (role 1) and prologues (role 2)
  std::vector<std::pair<size_t, int>> evdem;
  // lazily allocated readback scratch
  uint32_t* occ = nullptr;
  uint32_t* prof = nullptr;  // walkers per layer (the longest axis)
  double* mom_part = nullptr;
  size_t mom_part_n = 0;
  double* mom_out = nullptr;
  double* dref = nullptr;
  rwmi_batch* batch = nullptr;
  // two-way coupled particles
  bool dem = false;
  rwmi::DemArgs dem_host{};
  rwmi::DemArgs* dem_dev = nullptr;
};

struct rwmi_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<rwmi_domain*> members;
  bool dirty = true;
  // per precision group: device arrays of views and work maps
  struct Group {  // members of one precision, lattice layout and block size
    int prec;
    int inplace;
    int bs;
    std::vector<rwmi_domain*> doms;
    DomView* views = nullptr;
    int32_t* boff = nullptr;  // kRoles maps x (nd + 1)
    int blocks[kRoles] = {0, 0, 0};
  };
  std::vector<Group> groups;
  std::vector<void*> owned;
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  uint32_t gsteps = 0;
  int bs = 256;
  bool member_blocks = false;  // each member launches with its own block size
  int flags = rwmi::kFlagXcd;
};

namespace {

rwmi_status fail(rwmi_domain* d, rwmi_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (d) d->err = buf;
  g_err = buf;
  return st;
}

#define HIPCHK(d, call)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail((d), RWMI_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

void* dev_alloc(const Alloc& al, size_t bytes) {
  if (bytes == 0) bytes = 16;
  bytes = (bytes + 255) & ~size_t(255);
  if (al.fa) return al.fa(bytes, al.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}
void dev_free(const Alloc& al, void* p) {
  if (!p) return;
  if (al.ff) al.ff(p, al.ctx);
  else (void)hipFree(p);
}

template <typename T>
rwmi_status alloc_into(rwmi_domain* d, T*& out, size_t bytes) {
  void* p = dev_alloc(d->al, bytes);
  if (!p) return fail(d, RWMI_ENOMEM, "device allocation of %zu bytes failed", bytes);
  d->owned.push_back(p);
  out = (T*)p;
  return RWMI_OK;
}

void release(rwmi_domain* d, void* p) {
  if (!p) return;
  auto it = std::find(d->owned.begin(), d->owned.end(), p);
  if (it != d->owned.end()) d->owned.erase(it);
  dev_free(d->al, p);
}

int64_t mask_blocks(const rwmi_domain_desc& s, int32_t mb[3]) {
  int64_t t = 1;
  for (int a = 0; a < 3; ++a) {
    mb[a] = (s.n[a] + rwmi::kMaskBlock - 1) / rwmi::kMaskBlock;
    t *= mb[a];
  }
  return t;
}

rwmi_status upload_view(rwmi_domain* d) {
  HIPCHK(d, hipMemcpyAsync(d->dv, &d->hv, sizeof(DomView), hipMemcpyHostToDevice, d->stream));
  return RWMI_OK;
}

// Fluid cull words per table slot: one per fluid block at the smallest block
// size.
int64_t fcull_words(int64_t N) { return (N + 127) / 128; }

int blocks_for(int64_t n, int bs) { return (int)std::max<int64_t>(1, (n + bs - 1) / bs); }

// Blocks per role of one domain at bs threads per block: walkers, prologue
// (whenever there are particles: poses, one thread per fluid block for its
// cull word, and one per coarse block for the walker cull mask when there are
// walkers), fluid.
void role_blocks(const rwmi_domain* d, int bs, int b[kRoles]) {
  const int64_t nmb = (int64_t)d->hv.mb[0] * d->hv.mb[1] * d->hv.mb[2];
  const int64_t nfb = (d->hv.N + bs - 1) / bs;
  b[kRoleWalk] = d->hv.nw > 0 ? blocks_for(d->hv.nw, bs) : 0;
  b[kRolePro] = d->hv.np > 0 ? blocks_for(std::max<int64_t>(d->hv.nw > 0 ? nmb : 0, nfb), bs) : 0;
  b[kRoleFluid] = blocks_for(d->hv.N, bs);
}

// Blocks per role of launch j of a group of n steps (j = -1: the
// prologue-only launch that opens the group).
void launch_roles(const int b[kRoles], int j, uint32_t n, int nb[kRoles]) {
  const int64_t nn = (int64_t)n;
  nb[kRoleWalk] = j >= 1 ? b[kRoleWalk] : 0;
  nb[kRolePro] = (j == -1 || (j >= 0 && j < nn - 1)) ? b[kRolePro] : 0;
  nb[kRoleFluid] = (j >= 0 && j < nn) ? b[kRoleFluid] : 0;
}

rwmi_status upload_workmaps(rwmi_domain* d) {
  int b[kRoles];
  role_blocks(d, d->bs, b);
  int32_t h[2 * kRoles];
  for (int k = 0; k < kRoles; ++k) {
    h[2 * k] = 0;
    h[2 * k + 1] = b[k];
  }
  HIPCHK(d, hipMemcpyAsync(d->dboff, h, sizeof h, hipMemcpyHostToDevice, d->stream));
  HIPCHK(d, hipStreamSynchronize(d->stream));  // h lives on this stack frame
  return RWMI_OK;
}

void drop_graph(rwmi_domain* d) {
  if (d->gexec) {
    // no launch of the executable graph may still be in flight
    (void)hipStreamSynchronize(d->stream);
    (void)hipGraphExecDestroy(d->gexec);
    d->gexec = nullptr;
    d->gsteps = 0;
  }
}

// Upload the particle table and control points (once, before seeding or the
// first step).
rwmi_status finalize_particles(rwmi_domain* d) {
  if (d->particles_uploaded) return RWMI_OK;
  const int np = (int)d->parts.size();
  std::vector<DevParticle> hp(std::max(np, 1));
  std::vector<double> ctrl;
  for (int p = 0; p < np; ++p) {
    const HostParticle& q = d->parts[p];
    DevParticle& r = hp[p];
    std::memset(&r, 0, sizeof r);
    const int nc = (int)q.k.size();
    double K = 0.0, bmax = 0.0;
    for (int i = 0; i < nc; ++i) {
      K = K + q.k[i];
      const double* b = &q.b[3 * i];
      const double rr = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      if (rr > bmax) bmax = rr;
    }
    r.rb = bmax + std::sqrt(K);
    r.epscut2 = (r.rb + 0.75) * (r.rb + 0.75);
    r.shell2 = (std::sqrt(K) + 0.75) * (std::sqrt(K) + 0.75);
    r.maskr = r.rb + 0.5;
    for (int a = 0; a < 3; ++a) {
      r.c0[a] = q.c0[a];
      r.amp[a] = q.amp[a];
      r.vel[a] = q.vel[a];
    }
    r.period = q.period;
    r.phase = q.phase;
    r.motion = q.motion;
    r.nc = nc;
    r.ctrl0 = (int)(ctrl.size() / 4);
    for (int i = 0; i < nc; ++i) {
      ctrl.push_back(q.b[3 * i]);
      ctrl.push_back(q.b[3 * i + 1]);
      ctrl.push_back(q.b[3 * i + 2]);
      ctrl.push_back(q.k[i]);
    }
  }
  DevParticle* dp;
  double* dc;
  float* dcf;
  double* dpose;
  rwmi_status st;
  std::vector<float> ctrl_f(ctrl.begin(), ctrl.end());
  if ((st = alloc_into(d, dp, sizeof(DevParticle) * hp.size())) != RWMI_OK) return st;
  if ((st = alloc_into(d, dc, sizeof(double) * std::max<size_t>(ctrl.size(), 4))) != RWMI_OK) return st;
  if ((st = alloc_into(d, dcf, sizeof(float) * std::max<size_t>(ctrl.size(), 4))) != RWMI_OK) return st;
  if ((st = alloc_into(d, dpose, sizeof(double) * 6 * rwmi::kPoseRec * std::max(np, 1))) != RWMI_OK) return st;
  float* dsph;
  if ((st = alloc_into(d, dsph, sizeof(float) * 12 * std::max(np, 1))) != RWMI_OK) return st;
  HIPCHK(d, hipMemcpyAsync(dp, hp.data(), sizeof(DevParticle) * hp.size(), hipMemcpyHostToDevice, d->stream));
  if (!ctrl.empty()) {
    HIPCHK(d, hipMemcpyAsync(dc, ctrl.data(), sizeof(double) * ctrl.size(), hipMemcpyHostToDevice, d->stream));
    HIPCHK(d, hipMemcpyAsync(dcf, ctrl_f.data(), sizeof(float) * ctrl_f.size(), hipMemcpyHostToDevice, d->stream));
  }
  HIPCHK(d, hipStreamSynchronize(d->stream));  // host vectors go out of scope
  d->hv.parts = dp;
  d->hv.ctrl = dc;
  d->hv.ctrl_f = dcf;
  for (int k = 0; k < 3; ++k) {
    d->hv.ctrlr[k] = dc;  // nothing rotates unless coupled particles are set up
    d->hv.ctrlr_f[k] = dcf;
    d->hv.pose[k] = dpose + 2 * rwmi::kPoseRec * std::max(np, 1) * k;
    d->hv.sph[k] = dsph + 4 * std::max(np, 1) * k;
  }
  d->hv.np = np;
  if (np > 0) {
    unsigned long long* mask;
    int32_t mb[3];
    const int64_t nmb = mask_blocks(d->desc, mb);
    if ((st = alloc_into(d, mask, 24 * nmb)) != RWMI_OK) return st;
    for (int k = 0; k < 3; ++k) d->hv.mask[k] = mask + nmb * k;
    // fluid cull words for the smallest block size
    unsigned long long* fcull;
    const int64_t nfw = fcull_words(d->hv.N);
    if ((st = alloc_into(d, fcull, 24 * nfw)) != RWMI_OK) return st;
    for (int k = 0; k < 3; ++k) d->hv.fcull[k] = fcull + nfw * k;
  }
  d->particles_uploaded = true;
  if ((st = upload_view(d)) != RWMI_OK) return st;
  return upload_workmaps(d);
}

// Timing events: no host reads device data through them, so they skip the
// system-scope cache write-back and invalidation a default event performs
// (which also stalls the stream around each record).
struct TimedWindowState {
  size_t ev;
  uint32_t launches, fluid, walkers;
};

hipEvent_t take_event(rwmi_domain* d) {
  if (d->evused == d->evpool.size()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    d->evpool.push_back(e);
  }
  return d->evpool[d->evused++];
}

// Regroup the walkers before launch j of a group of n?  Every sort_every
// launches inside a group, and at its start when due (always at the start of
// a captured group, whose replays cannot consult the host).
bool sort_before(const rwmi_domain* d, uint32_t j, uint32_t n, bool capturing) {
  const uint32_t S = (uint32_t)d->sort_every;
  if (S == 0 || d->hv.nw == 0 || j >= n || j % S != 0) return false;
  // seeded walkers come in id order, scattered over the lattice: the first
  // group regroups them at its start
  return j > 0 || capturing || d->sorted_at == kNeverSorted || d->steps - d->sorted_at >= S;
}

// A launch group of n coupled steps for one domain: the prologue-only launch
// of step t0, then launches j = 0..n of the fused step kernel on the domain
// stream (launch j: fluid of t0 + j for j < n, prologue of t0 + j + 1 for
// j < n - 1, walkers of t0 + j - 1 for j >= 1), with the walker regrouping
// between launches, then the device step counter advances by n.  With
// `record`, HIP events bracket windows of timing_every consecutive step
// launches (j >= 0); a window closes early before a regrouping and at the
// end of the group, so it times step launches only.
rwmi_status enqueue_group_dem(rwmi_domain* d, uint32_t n, bool record, bool capturing);

// Flags of a domain's step launches: the caller's, plus the coupling's
// (interpolated bounce-back reads every step's densities).
int launch_flags(const rwmi_domain* d) {
  return d->flags | (d->hv.ibb ? rwmi::kFlagIbb | rwmi::kFlagDensity : 0);
}

rwmi_status enqueue_group(rwmi_domain* d, uint32_t n, bool record, bool capturing) {
  if (d->dem) return enqueue_group_dem(d, n, record, capturing);
  int b[kRoles];
  role_blocks(d, d->bs, b);
  hipStream_t A = d->stream;
  bool open = false;
  TimedWindowState win{};
  auto close_window = [&]() -> rwmi_status {
    if (!open) return RWMI_OK;
    HIPCHK(d, hipEventRecord(d->evpool[win.ev + 1], A));
    d->evrec.push_back({win.ev, win.launches, win.fluid, win.walkers});
    open = false;
    return RWMI_OK;
  };
  for (int j = -1; j <= (int)n; ++j) {
    if (j >= 0 && sort_before(d, (uint32_t)j, n, capturing)) {
      if (close_window() != RWMI_OK) return RWMI_EDEVICE;
      HIPCHK(d, rwmi::launch_sort(d->prec, d->dv, 0, d->hv.nw, d->sort, A));
      if (!capturing) d->sorted_at = d->steps + (uint32_t)j;
    }
    rwmi::StepArgs a{};
    a.views = d->dv;
    a.boff = d->dboff;
    a.nd = 1;
    launch_roles(b, j, n, a.nb);
    // the group's last fluid step also stores the densities for read-outs
    a.flags = launch_flags(d) | (j == (int)n - 1 ? rwmi::kFlagDensity : 0);
    a.inplace = d->hv.inplace;
    a.j = j;
    if (a.nb[0] + a.nb[1] + a.nb[2] == 0) continue;
    const bool timed = record && j >= 0;
    if (timed && !open) {
      win = TimedWindowState{d->evused, 0, 0, 0};
      hipEvent_t e0 = take_event(d), e1 = take_event(d);
      if (!e0 || !e1) return fail(d, RWMI_EDEVICE, "hipEventCreate failed");
      HIPCHK(d, hipEventRecord(e0, A));
      open = true;
    }
    if (d->hv.ibb && a.nb[kRoleFluid] > 0)
      HIPCHK(d, rwmi::launch_ibb_links(d->prec, d->dv, 0, j, false, (unsigned)a.nb[kRoleFluid], A));
    HIPCHK(d, rwmi::launch_step(d->prec, d->bs, a, A));
    if (timed) {
      win.launches += 1;
      win.fluid += a.nb[kRoleFluid] > 0 ? 1u : 0u;
      win.walkers += a.nb[kRoleWalk] > 0 ? 1u : 0u;
      if (win.launches == d->timing_every && close_window() != RWMI_OK) return RWMI_EDEVICE;
    }
  }
  if (close_window() != RWMI_OK) return RWMI_EDEVICE;
  HIPCHK(d, rwmi::launch_advance(d->dv, 1, n, A));
  return RWMI_OK;
}

// A launch group of n steps with two-way coupled particles.  The poses of a
// step are known only once the particle update of the previous step has run,
// so each step is three launches: the fused launch j (walkers of t0 + j - 1
// and fluid of t0 + j, which accumulates the hydrodynamic force), the
// particle update of t0 + j (poses and control points of t0 + j + 1) and the
// prologue of t0 + j + 1 (cull masks at those poses); then the walkers of
// the last step.  With `record`, an event pair brackets each launch: the
// step launches as one-launch windows of the step record, the particle
// updates and prologues in their own record.
rwmi_status enqueue_group_dem(rwmi_domain* d, uint32_t n, bool record, bool capturing) {
  int b[kRoles];
  role_blocks(d, d->bs, b);
  hipStream_t A = d->stream;
  size_t ev = 0;
  auto open = [&]() -> rwmi_status {
    if (!record) return RWMI_OK;
    ev = d->evused;
    hipEvent_t e0 = take_event(d), e1 = take_event(d);
    if (!e0 || !e1) return fail(d, RWMI_EDEVICE, "hipEventCreate failed");
    HIPCHK(d, hipEventRecord(e0, A));
    return RWMI_OK;
  };
  auto close = [&]() -> rwmi_status {
    if (!record) return RWMI_OK;
    HIPCHK(d, hipEventRecord(d->evpool[ev + 1], A));
    return RWMI_OK;
  };
  for (int j = 0; j <= (int)n; ++j) {
    if (sort_before(d, (uint32_t)j, n, capturing)) {
      HIPCHK(d, rwmi::launch_sort(d->prec, d->dv, 0, d->hv.nw, d->sort, A));
      if (!capturing) d->sorted_at = d->steps + (uint32_t)j;
    }
    rwmi::StepArgs a{};
    a.views = d->dv;
    a.boff = d->dboff;
    a.nd = 1;
    a.nb[kRoleWalk] = j >= 1 ? b[kRoleWalk] : 0;
    a.nb[kRolePro] = 0;
    a.nb[kRoleFluid] = j < (int)n ? b[kRoleFluid] : 0;
    a.flags = launch_flags(d) | rwmi::kFlagDem | (j == (int)n - 1 ? rwmi::kFlagDensity : 0);
    a.inplace = d->hv.inplace;
    a.j = j;
    if (a.nb[kRoleWalk] + a.nb[kRoleFluid] > 0) {
      if (open() != RWMI_OK) return RWMI_EDEVICE;
      if (d->hv.ibb && a.nb[kRoleFluid] > 0)
        HIPCHK(d, rwmi::launch_ibb_links(d->prec, d->dv, 0, j, true, (unsigned)a.nb[kRoleFluid], A));
      HIPCHK(d, rwmi::launch_step(d->prec, 256, a, A));
      if (close() != RWMI_OK) return RWMI_EDEVICE;
      if (record)
        d->evrec.push_back({ev, 1u, a.nb[kRoleFluid] > 0 ? 1u : 0u, a.nb[kRoleWalk] > 0 ? 1u : 0u});
    }
    if (j == (int)n) break;
    if (open() != RWMI_OK) return RWMI_EDEVICE;
    HIPCHK(d, rwmi::launch_dem(d->dv, d->dem_dev, j, A));
    if (close() != RWMI_OK) return RWMI_EDEVICE;
    if (record) d->evdem.push_back({ev, 1});
    a.nb[kRoleWalk] = 0;
    a.nb[kRolePro] = b[kRolePro];
    a.nb[kRoleFluid] = 0;
    a.flags = launch_flags(d) | rwmi::kFlagDem;
    if (open() != RWMI_OK) return RWMI_EDEVICE;
    HIPCHK(d, rwmi::launch_step(d->prec, 256, a, A));
    if (close() != RWMI_OK) return RWMI_EDEVICE;
    if (record) d->evdem.push_back({ev, 2});
  }
  HIPCHK(d, rwmi::launch_advance(d->dv, 1, n, A));
  return RWMI_OK;
}

// ---- set-up of coupled particles (host arithmetic: once per particle)
// Metaball value and gradient (Eq. 3, Eq. 17) at offset x from the reference
// point, in control-point order.
double host_M(const HostParticle& q, const double x[3]) {
  double M = 0.0;
  for (size_t i = 0; i < q.k.size(); ++i) {
    const double rx = x[0] - q.b[3 * i], ry = x[1] - q.b[3 * i + 1], rz = x[2] - q.b[3 * i + 2];
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == 0.0) return INFINITY;
    M = M + q.k[i] / r2;
  }
  return M;
}
void host_grad(const HostParticle& q, const double x[3], double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  for (size_t i = 0; i < q.k.size(); ++i) {
    const double r[3] = {x[0] - q.b[3 * i], x[1] - q.b[3 * i + 1], x[2] - q.b[3 * i + 2]};
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double f = (-2.0 * q.k[i]) / (r2 * r2);
    for (int a = 0; a < 3; ++a) g[a] = g[a] + f * r[a];
  }
}
// Solid fraction of the cell of size h centred at x: 1/2 + the distance
// estimate 2 M (sqrt M - 1) / |grad M| in cell units, clamped to [0, 1].
double host_cell_fraction(const HostParticle& q, const double x[3], double h) {
  const double M = host_M(q, x);
  if (M == INFINITY) return 1.0;
  double g[3];
  host_grad(q, x, g);
  const double gn = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  double e;
  if (gn == 0.0) e = M >= 1.0 ? 1.0 : 0.0;
  else e = 0.5 + (((2.0 * M) * (std::sqrt(M) - 1.0)) / gn) / h;
  if (!(e > 0.0)) e = 0.0;
  if (e > 1.0) e = 1.0;
  return e;
}
// Mass, centre of mass (offset from the reference point) and inertia tensor
// of a metaball of density rho: cells of size rb/24 over the cube
// [-rb - h, rb + h]^3, weighted by their solid fractions, summed z, y, x.
void host_mass_properties(const HostParticle& q, double rb, double rho, double* mass, double com[3],
                          double I[3][3]) {
  const int G = 50;
  const double h = rb / 24.0;
  double V = 0.0, S[3] = {0.0, 0.0, 0.0};
  for (int iz = 0; iz < G; ++iz)
    for (int iy = 0; iy < G; ++iy)
      for (int ix = 0; ix < G; ++ix) {
        const double x[3] = {((double)(ix - 25) + 0.5) * h, ((double)(iy - 25) + 0.5) * h,
                             ((double)(iz - 25) + 0.5) * h};
        const double e = host_cell_fraction(q, x, h);
        V = V + e;
        for (int a = 0; a < 3; ++a) S[a] = S[a] + e * x[a];
      }
  for (int a = 0; a < 3; ++a) com[a] = S[a] / V;
  double Q[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int iz = 0; iz < G; ++iz)
    for (int iy = 0; iy < G; ++iy)
      for (int ix = 0; ix < G; ++ix) {
        const double x[3] = {((double)(ix - 25) + 0.5) * h, ((double)(iy - 25) + 0.5) * h,
                             ((double)(iz - 25) + 0.5) * h};
        const double e = host_cell_fraction(q, x, h);
        const double r[3] = {x[0] - com[0], x[1] - com[1], x[2] - com[2]};
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) Q[a][c] = Q[a][c] + e * (r[a] * r[c]);
      }
  const double h3 = (h * h) * h;
  *mass = (rho * V) * h3;
  const double tr = (Q[0][0] + Q[1][1]) + Q[2][2];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) I[a][c] = (rho * h3) * ((a == c ? tr : 0.0) - Q[a][c]);
}
bool host_inv3(const double A[3][3], double X[3][3]) {
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double det = (A[0][0] * c00 + A[0][1] * c01) + A[0][2] * c02;
  if (det == 0.0 || !std::isfinite(det)) return false;
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
// w = R I_b^-1 R^T L for the unit quaternion q.
void host_omega(const double q[4], const double* Ibinv, const double L[3], double w[3]) {
  const double qw = q[0], x = q[1], y = q[2], z = q[3];
  double R[3][3];
  R[0][0] = 1.0 - 2.0 * (y * y + z * z);
  R[0][1] = 2.0 * (x * y - qw * z);
  R[0][2] = 2.0 * (x * z + qw * y);
  R[1][0] = 2.0 * (x * y + qw * z);
  R[1][1] = 1.0 - 2.0 * (x * x + z * z);
  R[1][2] = 2.0 * (y * z - qw * x);
  R[2][0] = 2.0 * (x * z - qw * y);
  R[2][1] = 2.0 * (y * z + qw * x);
  R[2][2] = 1.0 - 2.0 * (x * x + y * y);
  double yv[3], zv[3];
  for (int a = 0; a < 3; ++a) yv[a] = (R[0][a] * L[0] + R[1][a] * L[1]) + R[2][a] * L[2];
  for (int a = 0; a < 3; ++a) zv[a] = (Ibinv[3 * a] * yv[0] + Ibinv[3 * a + 1] * yv[1]) + Ibinv[3 * a + 2] * yv[2];
  for (int a = 0; a < 3; ++a) w[a] = (R[a][0] * zv[0] + R[a][1] * zv[1]) + R[a][2] * zv[2];
}

bool valid_prec(int p) { return p >= RWMI_FP64 && p <= RWMI_BF16_STORE; }

}  // namespace

extern "C" {

uint64_t rwmi_footprint_bytes(const rwmi_domain_desc* s, uint32_t n_particles, uint32_t n_ctrl_total,
                              uint64_t n_walkers) {
  if (!s) return 0;
  const uint64_t N = (uint64_t)s->n[0] * s->n[1] * s->n[2];
  const int p = s->precision;
  int32_t mb[3];
  const uint64_t nmb = (uint64_t)mask_blocks(*s, mb);
  uint64_t b = 0;
  b += (default_inplace(*s) ? 1 : 2) * rwmi::f_elems((int64_t)N) * elem_size(p) + 7 * N * u_size(p);
  b += sizeof(DomView) + 64 + 16;
  b += n_particles * sizeof(DevParticle) + 48 * n_ctrl_total + (288 + 48) * n_particles +
       (n_particles ? 24 * nmb + 24 * (uint64_t)fcull_words((int64_t)N) : 0);
  // walkers: cell, offsets, images, id and slot maps; sort scratch (bin, rank
  // and a second copy of the walker record) and the bin counts
  b += n_walkers * (4 + 3 * off_size(p) + 12 + 8);
  b += n_walkers * (8 + 4 + 3 * off_size(p) + 12 + 4) + 68 * nmb + 4 * (nmb / 4096 + 1);
  b += 4 * N;  // occupancy
  b += 8 * (6 * ((n_walkers + 4095) / 4096) + 12 * ((N + 4095) / 4096) + 64);
  return b;
}

rwmi_status rwmi_create_domain(const rwmi_domain_desc* s, rwmi_domain** out) {
  if (!s || !out) return fail(nullptr, RWMI_EINVAL, "null argument");
  *out = nullptr;
  for (int a = 0; a < 3; ++a) {
    if (s->n[a] < 1) return fail(nullptr, RWMI_EINVAL, "n[%d] = %d must be >= 1", a, s->n[a]);
    if (s->bc[a] != RWMI_BC_PERIODIC && s->bc[a] != RWMI_BC_WALL)
      return fail(nullptr, RWMI_EINVAL, "bc[%d] = %d unknown", a, s->bc[a]);
    if (s->bc[a] == RWMI_BC_WALL && s->n[a] < 3)
      return fail(nullptr, RWMI_EINVAL, "a wall axis needs at least 3 nodes (axis %d)", a);
  }
  const int64_t N = (int64_t)s->n[0] * s->n[1] * s->n[2];
  if (N > rwmi::kMaxNodes)
    return fail(nullptr, RWMI_EINVAL, "lattice of %lld nodes too large (at most %lld: 32-bit element indices)",
                (long long)N, (long long)rwmi::kMaxNodes);
  if (!(s->tau > 0.5)) return fail(nullptr, RWMI_EINVAL, "tau = %g must be > 0.5", s->tau);
  if (!(s->diffusivity >= 0.0)) return fail(nullptr, RWMI_EINVAL, "diffusivity must be >= 0");
  if (!valid_prec(s->precision)) return fail(nullptr, RWMI_EINVAL, "precision %d unknown", s->precision);
  if ((s->alloc == nullptr) != (s->free == nullptr))
    return fail(nullptr, RWMI_EINVAL, "alloc and free callbacks must be given together");
  {
    const hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return fail(nullptr, RWMI_EDEVICE, "hipSetDevice(%d) failed: %s", s->device, hipGetErrorString(e));
  }

  rwmi_domain* d = new rwmi_domain();
  d->desc = *s;
  d->prec = s->precision;
  d->device = s->device;
  d->al.fa = s->alloc;
  d->al.ff = s->free;
  d->al.ctx = s->alloc_ctx;
  if (s->stream) {
    d->stream = (hipStream_t)s->stream;
  } else {
    if (hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking) != hipSuccess) {
      delete d;
      return fail(nullptr, RWMI_EDEVICE, "hipStreamCreate failed");
    }
    d->own_stream = true;
  }
  DomView& v = d->hv;
  std::memset(&v, 0, sizeof v);
  for (int a = 0; a < 3; ++a) {
    v.n[a] = s->n[a];
    v.bc[a] = s->bc[a];
  }
  mask_blocks(*s, v.mb);
  v.dx = rwmi::make_fastdiv(s->n[0]);
  v.dy = rwmi::make_fastdiv(s->n[1]);
  v.dmx = rwmi::make_fastdiv(v.mb[0]);
  v.dmy = rwmi::make_fastdiv(v.mb[1]);
  v.N = N;
  v.prec = d->prec;
  v.inplace = default_inplace(*s) ? 1 : 0;
  const double rho0 = s->rho0 > 0 ? s->rho0 : 1.0;
  v.tau = s->tau;
  v.omega = 1.0 / s->tau;
  v.tm = s->tau - 0.5;
  v.cfree = 1.0 - 0.5 * v.omega;
  v.rho0 = rho0;
  v.sD = std::sqrt(2.0 * s->diffusivity);
  v.omega_f = (float)v.omega;
  v.tm_f = (float)v.tm;
  v.cfree_f = (float)v.cfree;
  v.rho0_f = (float)rho0;
  v.sD_f = (float)v.sD;
  v.has_force = 0;
  for (int i = 0; i < rwmi::kQ; ++i)
    v.eF_f[i] = (float)((double)rwmi::kEx[i] * s->force[0] + (double)rwmi::kEy[i] * s->force[1] +
                        (double)rwmi::kEz[i] * s->force[2]);
  for (int a = 0; a < 3; ++a) {
    v.F[a] = s->force[a];
    v.F_f[a] = (float)s->force[a];
    v.halfF_f[a] = (float)(0.5 * s->force[a]);
    if (s->force[a] != 0.0) v.has_force = 1;
    for (int c = 0; c < 3; ++c) {
      v.wu[a][0][c] = s->wall_u_lo[a][c];
      v.wu[a][1][c] = s->wall_u_hi[a][c];
      v.wu_f[a][0][c] = (float)s->wall_u_lo[a][c];
      v.wu_f[a][1][c] = (float)s->wall_u_hi[a][c];
    }
  }
  v.key0 = (uint32_t)s->seed;
  v.key1 = (uint32_t)(s->seed >> 32);
  v.max_bisect = 200;

  rwmi_status st = RWMI_OK;
  void *fA, *fB, *ub;
  uint64_t* tstep;
  unsigned long long* cnt;
  fB = nullptr;
  if ((st = alloc_into(d, fA, rwmi::f_elems(N) * elem_size(d->prec))) != RWMI_OK ||
      (!v.inplace && (st = alloc_into(d, fB, rwmi::f_elems(N) * elem_size(d->prec))) != RWMI_OK) ||
      (st = alloc_into(d, ub, 7 * (size_t)N * u_size(d->prec))) != RWMI_OK ||
      (st = alloc_into(d, tstep, 16)) != RWMI_OK || (st = alloc_into(d, cnt, 8 * rwmi::kCounters)) != RWMI_OK ||
      (st = alloc_into(d, d->dv, sizeof(DomView))) != RWMI_OK ||
      (st = alloc_into(d, d->dboff, sizeof(int32_t) * 2 * kRoles)) != RWMI_OK) {
    rwmi_destroy_domain(d);
    return fail(nullptr, st, "%s", g_err.c_str());
  }
  v.fA = fA;
  v.fB = fB;
  // two velocity buffers of 3 U per node, then the densities
  v.u[0] = ub;
  v.u[1] = (char*)ub + 3 * (size_t)N * u_size(d->prec);
  v.rho = (char*)ub + 6 * (size_t)N * u_size(d->prec);
  v.tstep = tstep;
  v.counters = cnt;
  uint64_t zeros[rwmi::kCounters] = {0};
  if (hipMemcpyAsync(tstep, zeros, 16, hipMemcpyHostToDevice, d->stream) != hipSuccess ||
      hipMemcpyAsync(cnt, zeros, sizeof zeros, hipMemcpyHostToDevice, d->stream) != hipSuccess ||
      upload_view(d) != RWMI_OK || upload_workmaps(d) != RWMI_OK ||
      rwmi::launch_init(d->prec, d->dv, 0, N, s->u0, d->stream) != hipSuccess ||
      hipStreamSynchronize(d->stream) != hipSuccess) {
    rwmi_destroy_domain(d);
    return fail(nullptr, RWMI_EDEVICE, "device initialisation failed");
  }
  *out = d;
  return RWMI_OK;
}

void rwmi_destroy_domain(rwmi_domain* d) {
  if (!d) return;
  (void)hipSetDevice(d->device);
  // a domain still in a batch leaves it first, so that the batch never holds
  // a pointer to freed memory (whatever order a caller destroys them in)
  if (d->batch) (void)rwmi_batch_remove(d->batch, d);
  if (d->stream) (void)hipStreamSynchronize(d->stream);
  drop_graph(d);
  for (hipEvent_t e : d->evpool) (void)hipEventDestroy(e);
  for (void* p : d->owned) dev_free(d->al, p);
  if (d->own_stream) (void)hipStreamDestroy(d->stream);
  delete d;
}

rwmi_status rwmi_add_metaball_particle(rwmi_domain* d, const rwmi_metaball_desc* p, int32_t* out_id) {
  if (!d || !p) return fail(d, RWMI_EINVAL, "null argument");
  if (d->seeded || d->stepped || d->particles_uploaded)
    return fail(d, RWMI_ESTATE, "particles must be added before seeding and stepping");
  if ((int)d->parts.size() >= RWMI_MAX_PARTICLES) return fail(d, RWMI_EINVAL, "at most %d particles", RWMI_MAX_PARTICLES);
  if (p->n_ctrl < 1 || p->n_ctrl > RWMI_MAX_CTRL || !p->offsets || !p->weights)
    return fail(d, RWMI_EINVAL, "n_ctrl = %d out of range", p->n_ctrl);
  if (p->motion < RWMI_MOTION_STATIC || p->motion > RWMI_MOTION_COUPLED) return fail(d, RWMI_EINVAL, "bad motion");
  if (p->motion == RWMI_MOTION_SINUSOID && !(p->period > 0.0)) return fail(d, RWMI_EINVAL, "period must be > 0");
  HostParticle h;
  h.b.assign(p->offsets, p->offsets + 3 * p->n_ctrl);
  h.k.assign(p->weights, p->weights + p->n_ctrl);
  for (double k : h.k)
    if (!(k > 0.0)) return fail(d, RWMI_EINVAL, "control-point weights must be > 0");
  for (int a = 0; a < 3; ++a) {
    h.c0[a] = p->centre[a];
    h.amp[a] = p->amplitude[a];
    h.vel[a] = p->velocity[a];
  }
  h.period = p->motion == RWMI_MOTION_SINUSOID ? p->period : 1.0;
  h.phase = p->phase;
  h.motion = p->motion;
  d->parts.push_back(h);
  if (out_id) *out_id = (int32_t)d->parts.size() - 1;
  return RWMI_OK;
}

rwmi_status rwmi_seed_walkers(rwmi_domain* d, const rwmi_seed_desc* s, uint64_t n, uint64_t* out_seeded) {
  if (!d || !s) return fail(d, RWMI_EINVAL, "null argument");
  if (out_seeded) *out_seeded = 0;
  if (d->seeded || d->stepped) return fail(d, RWMI_ESTATE, "walkers can be seeded once, before the first step");
  if (n > (uint64_t)INT32_MAX) return fail(d, RWMI_EINVAL, "too many walkers");
  if (s->kind < RWMI_SEED_UNIFORM || s->kind > RWMI_SEED_EXPLICIT) return fail(d, RWMI_EINVAL, "bad seed kind");
  if (s->kind == RWMI_SEED_EXPLICIT && n > 0 && !s->xyz) return fail(d, RWMI_EINVAL, "explicit seeding needs xyz");
  if (s->kind == RWMI_SEED_BAND && (s->band_axis < 0 || s->band_axis > 2 || !(s->band_hi > s->band_lo)))
    return fail(d, RWMI_EINVAL, "bad band");
  HIPCHK(d, hipSetDevice(d->device));
  rwmi_status st;
  if ((st = finalize_particles(d)) != RWMI_OK) return st;
  const size_t osz = off_size(d->prec);
  const int64_t nn = (int64_t)n;
  int32_t* tcell = nullptr;
  void* toff = nullptr;
  uint8_t* flag = nullptr;
  int32_t* pos = nullptr;
  double* dxyz = nullptr;
  std::vector<void*> tmp;
  auto cleanup = [&] {
    for (void* p : tmp) release(d, p);
  };
  if (nn > 0) {
    if ((st = alloc_into(d, tcell, 4 * nn)) != RWMI_OK) return st;
    tmp.push_back(tcell);
    if ((st = alloc_into(d, toff, 3 * osz * nn)) != RWMI_OK) return cleanup(), st;
    tmp.push_back(toff);
    if ((st = alloc_into(d, flag, nn)) != RWMI_OK) return cleanup(), st;
    tmp.push_back(flag);
    if ((st = alloc_into(d, pos, 4 * nn)) != RWMI_OK) return cleanup(), st;
    tmp.push_back(pos);
    if (s->kind == RWMI_SEED_EXPLICIT) {
      if ((st = alloc_into(d, dxyz, 24 * nn)) != RWMI_OK) return cleanup(), st;
      tmp.push_back(dxyz);
      if (hipMemcpyAsync(dxyz, s->xyz, 24 * nn, hipMemcpyHostToDevice, d->stream) != hipSuccess)
        return cleanup(), fail(d, RWMI_EDEVICE, "copy of explicit positions failed");
    }
  }
  const int attempts = s->kind == RWMI_SEED_EXPLICIT || s->remove_inside ? 1 : (s->max_attempts > 0 ? s->max_attempts : 64);
  std::vector<uint8_t> hflag(nn);
  if (nn > 0) {
    if (rwmi::launch_seed(d->prec, d->dv, 0, s->kind, s->centre, s->sigma, s->band_axis, s->band_lo, s->band_hi, dxyz,
                          nn, attempts, tcell, toff, flag, d->stream) != hipSuccess ||
        hipMemcpyAsync(hflag.data(), flag, nn, hipMemcpyDeviceToHost, d->stream) != hipSuccess ||
        hipStreamSynchronize(d->stream) != hipSuccess)
      return cleanup(), fail(d, RWMI_EDEVICE, "seeding kernel failed");
  }
  std::vector<int32_t> hpos(nn);
  int64_t m = 0;
  for (int64_t w = 0; w < nn; ++w) {
    hpos[w] = (int32_t)m;
    m += hflag[w];
  }
  // walker arrays of the final size
  int32_t *wcell, *wimg, *wid, *winv;
  void* woff;
  const int64_t m1 = std::max<int64_t>(m, 1);
  rwmi::SortScratch& sc = d->sort;
  sc.nbins = (int64_t)d->hv.mb[0] * d->hv.mb[1] * d->hv.mb[2];
  if ((st = alloc_into(d, wcell, 4 * m1)) != RWMI_OK || (st = alloc_into(d, woff, 3 * osz * m1)) != RWMI_OK ||
      (st = alloc_into(d, wimg, 12 * m1)) != RWMI_OK || (st = alloc_into(d, wid, 4 * m1)) != RWMI_OK ||
      (st = alloc_into(d, winv, 4 * m1)) != RWMI_OK || (st = alloc_into(d, sc.hist, 68 * sc.nbins + 4 * (sc.nbins / 4096 + 1))) != RWMI_OK ||
      (st = alloc_into(d, sc.bin, 4 * m1)) != RWMI_OK || (st = alloc_into(d, sc.rank, 4 * m1)) != RWMI_OK ||
      (st = alloc_into(d, sc.cell, 4 * m1)) != RWMI_OK || (st = alloc_into(d, sc.off, 3 * osz * m1)) != RWMI_OK ||
      (st = alloc_into(d, sc.img, 12 * m1)) != RWMI_OK || (st = alloc_into(d, sc.wid, 4 * m1)) != RWMI_OK)
    return cleanup(), st;
  d->hv.wcell = wcell;
  d->hv.woff = woff;
  d->hv.wimg = wimg;
  d->hv.wid = wid;
  d->hv.winv = winv;
  d->hv.nw = m;
  if ((st = upload_view(d)) != RWMI_OK) return cleanup(), st;
  if (m > 0) {
    if (hipMemcpyAsync(pos, hpos.data(), 4 * nn, hipMemcpyHostToDevice, d->stream) != hipSuccess ||
        rwmi::launch_seed_scatter(d->prec, d->dv, 0, nn, tcell, toff, flag, pos, m, d->stream) != hipSuccess ||
        rwmi::launch_ids_identity(d->dv, 0, m, d->stream) != hipSuccess)
      return cleanup(), fail(d, RWMI_EDEVICE, "seed scatter failed");
  }
  if (hipStreamSynchronize(d->stream) != hipSuccess) return cleanup(), fail(d, RWMI_EDEVICE, "seeding failed");
  cleanup();
  for (int a = 0; a < 3; ++a) d->ref[a] = s->ref[a];
  d->seeded = true;
  if ((st = upload_workmaps(d)) != RWMI_OK) return st;
  drop_graph(d);
  if (out_seeded) *out_seeded = (uint64_t)m;
  if (m < nn && !s->remove_inside)
    return fail(d, RWMI_ESEED, "%lld of %lld walkers found no admissible position", (long long)(nn - m), (long long)nn);
  return RWMI_OK;
}

rwmi_status rwmi_step(rwmi_domain* d, uint32_t n_steps) {
  if (!d) return fail(d, RWMI_EINVAL, "null domain");
  if (d->batch) return fail(d, RWMI_ESTATE, "domain is stepped by its batch");
  HIPCHK(d, hipSetDevice(d->device));
  rwmi_status st;
  if ((st = finalize_particles(d)) != RWMI_OK) return st;
  d->stepped = true;
  uint32_t left = n_steps;
  if (d->use_graph && !d->timing && n_steps >= 2) {
    const uint32_t k = std::min<uint32_t>(n_steps, kGraphSteps);
    if (!d->gexec || d->gsteps != k) {
      drop_graph(d);
      hipGraph_t g;
      HIPCHK(d, hipStreamBeginCapture(d->stream, hipStreamCaptureModeThreadLocal));
      if ((st = enqueue_group(d, k, false, true)) != RWMI_OK) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(d->stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        return st;
      }
      HIPCHK(d, hipStreamEndCapture(d->stream, &g));
      hipError_t e = hipGraphInstantiate(&d->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(d, RWMI_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
      d->gsteps = k;
    }
    while (left >= d->gsteps) {
      HIPCHK(d, hipGraphLaunch(d->gexec, d->stream));
      left -= d->gsteps;
      if (d->sort_every > 0 && d->hv.nw > 0) d->sorted_at = d->steps;  // every replay sorts at its start
      d->steps += d->gsteps;
    }
  }
  if (left > 0) {
    if ((st = enqueue_group(d, left, d->timing, false)) != RWMI_OK) return st;
    d->steps += left;
  }
  return RWMI_OK;
}

rwmi_status rwmi_set_coupling(rwmi_domain* d, const rwmi_coupling_desc* c) {
  if (!d || !c) return fail(d, RWMI_EINVAL, "null argument");
  if (d->dem) return fail(d, RWMI_ESTATE, "coupling already set up");
  if (d->particles_uploaded || d->seeded || d->stepped)
    return fail(d, RWMI_ESTATE, "set up the coupling after adding the particles, before seeding and stepping");
  if (!(c->density > 0.0) || c->substeps < 1 || c->substeps > rwmi::kDemMaxSub || !(c->drive_period > 0.0) ||
      !(c->dilation_radius > 0.0) ||
      !(c->kn > 0.0) || c->kt < 0.0 || c->eta_n < 0.0 || c->eta_t < 0.0 || c->mu < 0.0)
    return fail(d, RWMI_EINVAL, "coupling parameters out of range");
  const int np = (int)d->parts.size();
  unsigned long long mask = 0ull;
  size_t nctrl = 0;
  for (int p = 0; p < np; ++p) {
    nctrl += d->parts[p].k.size();
    if (d->parts[p].motion == RWMI_MOTION_COUPLED) mask |= 1ull << p;
  }
  if (!mask) return fail(d, RWMI_EINVAL, "no particle has motion RWMI_MOTION_COUPLED");
  if (nctrl > (size_t)rwmi::kDemMaxCtrl)
    return fail(d, RWMI_EINVAL, "%zu control points in all; coupled particles allow at most %d", nctrl,
                rwmi::kDemMaxCtrl);
  HIPCHK(d, hipSetDevice(d->device));
  // mass properties; the centre of mass becomes each coupled particle's centre
  std::vector<double> state((size_t)rwmi::kDemState * np, 0.0);
  for (int p = 0; p < np; ++p) {
    HostParticle& q = d->parts[p];
    if (q.motion != RWMI_MOTION_COUPLED) continue;
    const int nc = (int)q.k.size();
    double K = 0.0, bmax = 0.0;
    for (int i = 0; i < nc; ++i) {
      K = K + q.k[i];
      const double* b = &q.b[3 * i];
      const double r = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      if (r > bmax) bmax = r;
    }
    const double sk = std::sqrt(K);
    if (!(sk > c->dilation_radius)) return fail(d, RWMI_EINVAL, "particle %d is thinner than the dilation radius", p);
    double mass, com[3], I[3][3], Iinv[3][3];
    host_mass_properties(q, bmax + sk, c->density, &mass, com, I);
    if (!host_inv3(I, Iinv)) return fail(d, RWMI_EINVAL, "particle %d has a singular inertia tensor", p);
    double bmax2 = 0.0;
    for (int i = 0; i < nc; ++i) {
      for (int a = 0; a < 3; ++a) q.b[3 * i + a] = q.b[3 * i + a] - com[a];
      const double* b = &q.b[3 * i];
      const double r = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      if (r > bmax2) bmax2 = r;
    }
    double* st = &state[(size_t)rwmi::kDemState * p];
    for (int a = 0; a < 3; ++a) {
      q.c0[a] = q.c0[a] + com[a];
      st[rwmi::kDc + a] = q.c0[a];
      st[rwmi::kDv + a] = q.vel[a];
    }
    st[rwmi::kDq] = 1.0;
    st[rwmi::kDm] = mass;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        st[rwmi::kDIb + 3 * a + b] = I[a][b];
        st[rwmi::kDIbinv + 3 * a + b] = Iinv[a][b];
      }
    st[rwmi::kDcin] = (sk / (sk - c->dilation_radius)) * (sk / (sk - c->dilation_radius));
    st[rwmi::kDrb] = bmax2 + sk;
  }
  rwmi_status st;
  if ((st = finalize_particles(d)) != RWMI_OK) return st;
  rwmi::DemArgs& A = d->dem_host;
  A.nsub = c->substeps;
  A.coupling = c->coupling ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    A.g[a] = c->gravity[a];
    A.drive_dir[a] = c->drive_direction[a];
  }
  A.drive_amp = c->drive_amplitude;
  A.drive_period = c->drive_period;
  A.kn = c->kn;
  A.kt = c->kt;
  A.eta_n = c->eta_n;
  A.eta_t = c->eta_t;
  A.mu = c->mu;
  A.Rs = c->dilation_radius;
  unsigned long long* acc;
  const size_t nct = std::max<size_t>(nctrl, 1);
  if ((st = alloc_into(d, A.state, sizeof(double) * state.size())) != RWMI_OK ||
      (st = alloc_into(d, A.xi, sizeof(double) * 3 * rwmi::kMaxParticles * rwmi::kMaxParticles)) != RWMI_OK ||
      (st = alloc_into(d, A.xiw, sizeof(double) * 3 * 6 * rwmi::kMaxParticles)) != RWMI_OK ||
      (st = alloc_into(d, A.xmask, sizeof(unsigned long long) * rwmi::kMaxParticles)) != RWMI_OK ||
      (st = alloc_into(d, acc, sizeof(unsigned long long) * 6 * np)) != RWMI_OK ||
      (st = alloc_into(d, d->dem_dev, sizeof(rwmi::DemArgs))) != RWMI_OK)
    return st;
  for (int k = 0; k < 3; ++k) {
    if ((st = alloc_into(d, A.ctrlr[k], sizeof(double) * 4 * nct)) != RWMI_OK ||
        (st = alloc_into(d, A.ctrlr_f[k], sizeof(float) * 4 * nct)) != RWMI_OK)
      return st;
    HIPCHK(d, hipMemcpyAsync(A.ctrlr[k], d->hv.ctrl, sizeof(double) * 4 * nctrl, hipMemcpyDeviceToDevice, d->stream));
    HIPCHK(d, hipMemcpyAsync(A.ctrlr_f[k], d->hv.ctrl_f, sizeof(float) * 4 * nctrl, hipMemcpyDeviceToDevice,
                             d->stream));
    d->hv.ctrlr[k] = A.ctrlr[k];
    d->hv.ctrlr_f[k] = A.ctrlr_f[k];
  }
  HIPCHK(d, hipMemsetAsync(A.xi, 0, sizeof(double) * 3 * rwmi::kMaxParticles * rwmi::kMaxParticles, d->stream));
  HIPCHK(d, hipMemsetAsync(A.xiw, 0, sizeof(double) * 3 * 6 * rwmi::kMaxParticles, d->stream));
  HIPCHK(d, hipMemsetAsync(A.xmask, 0, sizeof(unsigned long long) * rwmi::kMaxParticles, d->stream));
  HIPCHK(d, hipMemsetAsync(acc, 0, sizeof(unsigned long long) * 6 * np, d->stream));
  HIPCHK(d, hipMemcpyAsync(A.state, state.data(), sizeof(double) * state.size(), hipMemcpyHostToDevice, d->stream));
  HIPCHK(d, hipMemcpyAsync(d->dem_dev, &A, sizeof A, hipMemcpyHostToDevice, d->stream));
  d->hv.dem_mask = mask;
  d->hv.dem_acc = acc;
  d->dem = true;
  d->bs = 256;
  if ((st = upload_view(d)) != RWMI_OK || (st = upload_workmaps(d)) != RWMI_OK) return st;
  // poses and cull masks of the current step from the state
  HIPCHK(d, rwmi::launch_dem_tables(d->dv, d->dem_dev, d->stream));
  int b[kRoles];
  role_blocks(d, d->bs, b);
  rwmi::StepArgs a{};
  a.views = d->dv;
  a.boff = d->dboff;
  a.nd = 1;
  a.nb[kRolePro] = b[kRolePro];
  a.flags = launch_flags(d) | rwmi::kFlagDem;
  a.inplace = d->hv.inplace;
  a.j = -1;
  HIPCHK(d, rwmi::launch_step(d->prec, 256, a, d->stream));
  HIPCHK(d, hipStreamSynchronize(d->stream));  // `state` lives on this stack frame
  return RWMI_OK;
}

rwmi_status rwmi_set_fluid_coupling(rwmi_domain* d, int32_t scheme) {
  if (!d) return fail(d, RWMI_EINVAL, "null domain");
  if (scheme != RWMI_COUPLING_PSM && scheme != RWMI_COUPLING_IBB) return fail(d, RWMI_EINVAL, "unknown coupling %d", scheme);
  if (d->stepped || d->batch) return fail(d, RWMI_ESTATE, "the coupling is chosen before the first step");
  HIPCHK(d, hipSetDevice(d->device));
  rwmi_status st;
  if (scheme == RWMI_COUPLING_IBB) {
    if (d->hv.inplace && (st = rwmi_debug_set(d, RWMI_KEY_STREAMING, 1)) != RWMI_OK) return st;
    if (!d->hv.smap[0]) {
      uint8_t* sm;
      if ((st = alloc_into(d, sm, 2 * (size_t)d->hv.N)) != RWMI_OK) return st;
      HIPCHK(d, hipMemsetAsync(sm, 0, 2 * (size_t)d->hv.N, d->stream));
      d->hv.smap[0] = sm;
      d->hv.smap[1] = sm + d->hv.N;
      // lists of the solid nodes (any node can be one), for the link pass
      // of the next step
      uint32_t* nl;
      if ((st = alloc_into(d, nl, 4 * (2 * (size_t)d->hv.N + 2))) != RWMI_OK) return st;
      HIPCHK(d, hipMemsetAsync(nl + 2 * (size_t)d->hv.N, 0, 8, d->stream));
      d->hv.solid_list[0] = nl;
      d->hv.solid_list[1] = nl + d->hv.N;
      d->hv.solid_count = nl + 2 * (size_t)d->hv.N;
    }
    d->bs = 256;
  }
  d->hv.ibb = scheme == RWMI_COUPLING_IBB ? 1 : 0;
  drop_graph(d);
  if ((st = upload_view(d)) != RWMI_OK || (st = upload_workmaps(d)) != RWMI_OK) return st;
  if (d->dem) {  // the cull masks of the current step at this coupling's reach
    int b[kRoles];
    role_blocks(d, d->bs, b);
    rwmi::StepArgs a{};
    a.views = d->dv;
    a.boff = d->dboff;
    a.nd = 1;
    a.nb[kRolePro] = b[kRolePro];
    a.flags = launch_flags(d) | rwmi::kFlagDem;
    a.inplace = d->hv.inplace;
    a.j = -1;
    HIPCHK(d, rwmi::launch_step(d->prec, 256, a, d->stream));
  }
  HIPCHK(d, hipStreamSynchronize(d->stream));
  return RWMI_OK;
}

rwmi_status rwmi_read_particle_state(rwmi_domain* d, int32_t p, double* out) {
  if (!d || !out) return fail(d, RWMI_EINVAL, "null argument");
  if (!d->dem || p < 0 || p >= d->hv.np || !((d->hv.dem_mask >> p) & 1ull))
    return fail(d, RWMI_EINVAL, "particle %d is not a coupled particle", p);
  HIPCHK(d, hipSetDevice(d->device));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  HIPCHK(d, hipMemcpy(out, d->dem_host.state + (size_t)rwmi::kDemState * p, sizeof(double) * 32,
                      hipMemcpyDeviceToHost));
  return RWMI_OK;
}

rwmi_status rwmi_set_particle_motion(rwmi_domain* d, int32_t p, const double v[3], const double L[3]) {
  if (!d || !v || !L) return fail(d, RWMI_EINVAL, "null argument");
  if (!d->dem || p < 0 || p >= d->hv.np || !((d->hv.dem_mask >> p) & 1ull))
    return fail(d, RWMI_EINVAL, "particle %d is not a coupled particle", p);
  if (d->batch) return fail(d, RWMI_ESTATE, "domain is stepped by its batch");
  HIPCHK(d, hipSetDevice(d->device));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  double st[rwmi::kDemState];
  double* dst = d->dem_host.state + (size_t)rwmi::kDemState * p;
  HIPCHK(d, hipMemcpy(st, dst, sizeof st, hipMemcpyDeviceToHost));
  for (int a = 0; a < 3; ++a) {
    st[rwmi::kDv + a] = v[a];
    st[rwmi::kDL + a] = L[a];
  }
  host_omega(st + rwmi::kDq, st + rwmi::kDIbinv, st + rwmi::kDL, st + rwmi::kDw);
  HIPCHK(d, hipMemcpy(dst, st, sizeof st, hipMemcpyHostToDevice));
  HIPCHK(d, rwmi::launch_dem_tables(d->dv, d->dem_dev, d->stream));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  return RWMI_OK;
}

rwmi_status rwmi_synchronize(rwmi_domain* d) {
  if (!d) return fail(d, RWMI_EINVAL, "null domain");
  HIPCHK(d, hipSetDevice(d->device));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  return RWMI_OK;
}

rwmi_status rwmi_query_sizes(const rwmi_domain* d, uint64_t* n_nodes, uint64_t* n_walkers, uint64_t* step) {
  if (!d) return fail(nullptr, RWMI_EINVAL, "null domain");
  if (n_nodes) *n_nodes = (uint64_t)d->hv.N;
  if (n_walkers) *n_walkers = (uint64_t)d->hv.nw;
  if (step) *step = d->steps;
  return RWMI_OK;
}

rwmi_status rwmi_read_velocity(rwmi_domain* d, double* u, double* rho) {
  if (!d) return fail(d, RWMI_EINVAL, "null domain");
  HIPCHK(d, hipSetDevice(d->device));
  const int64_t N = d->hv.N;
  const size_t us = u_size(d->prec);
  // velocities of the last step (buffer of its parity), densities from the
  // group's last fluid step, which is the same step
  std::vector<unsigned char> h(3 * N * us), hr(N * us);
  const void* ub = d->hv.u[d->steps > 0 ? ((d->steps - 1) & 1) : 0];
  HIPCHK(d, hipMemcpyAsync(h.data(), ub, h.size(), hipMemcpyDeviceToHost, d->stream));
  HIPCHK(d, hipMemcpyAsync(hr.data(), d->hv.rho, hr.size(), hipMemcpyDeviceToHost, d->stream));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  auto at = [&](const std::vector<unsigned char>& b, int64_t k) -> double {
    return us == 8 ? ((const double*)b.data())[k] : (double)((const float*)b.data())[k];
  };
  for (int64_t i = 0; i < N; ++i) {
    if (u)
      for (int c = 0; c < 3; ++c) u[c * N + i] = at(h, 3 * i + c);
    if (rho) rho[i] = at(hr, i);
  }
  return RWMI_OK;
}

rwmi_status rwmi_read_walkers(rwmi_domain* d, int32_t* cell, double* off, int32_t* img) {
  if (!d) return fail(d, RWMI_EINVAL, "null domain");
  HIPCHK(d, hipSetDevice(d->device));
  const int64_t m = d->hv.nw;
  if (m == 0) return RWMI_OK;
  // slots hold walkers in any order; the output is in walker-id order
  std::vector<int32_t> wid(m), hc, hi;
  std::vector<double> hd;
  std::vector<float> hf;
  HIPCHK(d, hipMemcpyAsync(wid.data(), d->hv.wid, 4 * m, hipMemcpyDeviceToHost, d->stream));
  if (cell) {
    hc.resize(m);
    HIPCHK(d, hipMemcpyAsync(hc.data(), d->hv.wcell, 4 * m, hipMemcpyDeviceToHost, d->stream));
  }
  if (img) {
    hi.resize(3 * m);
    HIPCHK(d, hipMemcpyAsync(hi.data(), d->hv.wimg, 12 * m, hipMemcpyDeviceToHost, d->stream));
  }
  if (off) {
    if (d->prec == RWMI_FP64) {
      hd.resize(3 * m);
      HIPCHK(d, hipMemcpyAsync(hd.data(), d->hv.woff, 24 * m, hipMemcpyDeviceToHost, d->stream));
    } else {
      hf.resize(3 * m);
      HIPCHK(d, hipMemcpyAsync(hf.data(), d->hv.woff, 12 * m, hipMemcpyDeviceToHost, d->stream));
    }
  }
  HIPCHK(d, hipStreamSynchronize(d->stream));
  for (int64_t i = 0; i < m; ++i) {
    const int64_t w = wid[i];
    if (w < 0 || w >= m) return fail(d, RWMI_EDEVICE, "walker id map corrupt at slot %lld", (long long)i);
    if (cell) cell[w] = hc[i];
    for (int a = 0; a < 3; ++a) {
      if (img) img[a * m + w] = hi[a * m + i];
      if (off) off[a * m + w] = d->prec == RWMI_FP64 ? hd[a * m + i] : (double)hf[a * m + i];
    }
  }
  return RWMI_OK;
}

rwmi_status rwmi_read_distributions(rwmi_domain* d, double* f) {
  if (!d || !f) return fail(d, RWMI_EINVAL, "null argument");
  HIPCHK(d, hipSetDevice(d->device));
  const int64_t N = d->hv.N;
  double* tmp;
  rwmi_status st;
  if ((st = alloc_into(d, tmp, 8 * 19 * (size_t)N)) != RWMI_OK) return st;
  hipError_t e = rwmi::launch_read_f(d->prec, d->dv, 0, N, tmp, d->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(f, tmp, 8 * 19 * (size_t)N, hipMemcpyDeviceToHost, d->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
  release(d, tmp);
  if (e != hipSuccess) return fail(d, RWMI_EDEVICE, "read_distributions: %s", hipGetErrorString(e));
  return RWMI_OK;
}

rwmi_status rwmi_read_occupancy(rwmi_domain* d, uint32_t* ns) {
  if (!d || !ns) return fail(d, RWMI_EINVAL, "null argument");
  HIPCHK(d, hipSetDevice(d->device));
  rwmi_status st;
  if (!d->occ && (st = alloc_into(d, d->occ, 4 * (size_t)d->hv.N)) != RWMI_OK) return st;
  if (!d->hv.occ) {
    d->hv.occ = d->occ;
    if ((st = upload_view(d)) != RWMI_OK) return st;
    drop_graph(d);
  }
  HIPCHK(d, rwmi::launch_occupancy(d->dv, 0, d->occ, d->hv.N, d->hv.nw, d->stream));
  HIPCHK(d, hipMemcpyAsync(ns, d->occ, 4 * (size_t)d->hv.N, hipMemcpyDeviceToHost, d->stream));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  return RWMI_OK;
}

// The moments from the 32 doubles the final reduction wrote.
static void fill_moments(const rwmi_domain* d, const double h[32], rwmi_moments* out) {
  std::memset(out, 0, sizeof *out);
  const int64_t nw = d->hv.nw;
  uint64_t u64[rwmi::kCounters + 1];
  std::memcpy(u64, h + 18, sizeof u64);
  out->step = u64[rwmi::kCounters];
  out->n_walkers = (uint64_t)nw;
  for (int a = 0; a < 3; ++a) {
    out->sum[a] = h[a];
    out->sumsq[a] = h[3 + a];
    out->momentum[a] = h[7 + a];
    out->fluid_u[a] = h[13] > 0.0 ? h[10 + a] / h[13] : 0.0;
    out->particle_v[a] = h[17] > 0.0 ? h[14 + a] / h[17] : 0.0;
  }
  out->mass = h[6];
  out->solid_volume = h[17];
  out->type2 = u64[rwmi::kType2];
  out->type4 = u64[rwmi::kType4];
  out->bisect_fail = u64[rwmi::kBisectFail];
  out->refill_fallback = u64[rwmi::kRefillFallback];
  out->returned_to_origin = u64[rwmi::kReturned];
  out->wall_reflect = u64[rwmi::kWallReflect];
  out->near_surface = u64[rwmi::kNearSurface];
  out->contact_misses = u64[rwmi::kDemSkin];
}

rwmi_status rwmi_read_profile(rwmi_domain* d, int32_t axis, uint64_t* counts) {
  if (!d || !counts) return fail(d, RWMI_EINVAL, "null argument");
  if (axis < 0 || axis > 2) return fail(d, RWMI_EINVAL, "axis %d out of range", axis);
  HIPCHK(d, hipSetDevice(d->device));
  rwmi_status st;
  const int nmax = std::max(d->hv.n[0], std::max(d->hv.n[1], d->hv.n[2]));
  if (!d->prof && (st = alloc_into(d, d->prof, 4 * (size_t)nmax)) != RWMI_OK) return st;
  const int nl = d->hv.n[axis];
  std::vector<uint32_t> h(nl);
  HIPCHK(d, rwmi::launch_profile(d->dv, 0, axis, nl, d->hv.nw, d->prof, d->stream));
  HIPCHK(d, hipMemcpyAsync(h.data(), d->prof, 4 * (size_t)nl, hipMemcpyDeviceToHost, d->stream));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  for (int i = 0; i < nl; ++i) counts[i] = h[i];
  return RWMI_OK;
}

rwmi_status rwmi_read_moments(rwmi_domain* d, rwmi_moments* out) {
  if (!d || !out) return fail(d, RWMI_EINVAL, "null argument");
  HIPCHK(d, hipSetDevice(d->device));
  rwmi_status st;
  if ((st = finalize_particles(d)) != RWMI_OK) return st;
  const int64_t N = d->hv.N, nw = d->hv.nw;
  const size_t need = 6 * ((nw + 4095) / 4096) + 12 * ((N + 4095) / 4096) + 8;
  if (d->mom_part_n < need) {
    release(d, d->mom_part);
    d->mom_part = nullptr;
    if ((st = alloc_into(d, d->mom_part, 8 * need)) != RWMI_OK) return st;
    d->mom_part_n = need;
  }
  if (!d->mom_out && (st = alloc_into(d, d->mom_out, 8 * 32)) != RWMI_OK) return st;
  if (!d->dref && (st = alloc_into(d, d->dref, 8 * 4)) != RWMI_OK) return st;
  HIPCHK(d, hipMemcpyAsync(d->dref, d->ref, 24, hipMemcpyHostToDevice, d->stream));
  double* pw = d->mom_part;
  double* pn = d->mom_part + 6 * ((nw + 4095) / 4096);
  HIPCHK(d, rwmi::launch_moments(d->prec, d->dv, 0, N, nw, d->dref, pw, pn, d->mom_out, d->stream));
  double h[32];
  HIPCHK(d, hipMemcpyAsync(h, d->mom_out, sizeof h, hipMemcpyDeviceToHost, d->stream));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  fill_moments(d, h, out);
  return RWMI_OK;
}

// Same kernels and reduction order as rwmi_read_moments, with every buffer
// they need (output staging [0, 32), reference point [32, 36), walker
// partials from 64, node partials after them) in the library's per-GPU
// scratch array.  Nothing there has to start at zero: each reduction block
// writes its own partials and the final kernel writes every output word.
rwmi_status rwmi_read_moments_noalloc(rwmi_domain* d, rwmi_moments* out) {
  if (!d || !out) return fail(d, RWMI_EINVAL, "null argument");
  if (!d->particles_uploaded && !d->parts.empty())
    return fail(d, RWMI_ESTATE, "particles are uploaded by seeding or the first step; read moments after either");
  const int64_t N = d->hv.N, nw = d->hv.nw;
  const int64_t nbw = (nw + 4095) / 4096, nbn = (N + 4095) / 4096;
  const int64_t need = 64 + 6 * nbw + 12 * nbn;
  if (need > rwmi::kNoAllocDoubles)
    return fail(d, RWMI_EINVAL,
                "the allocation-free read-out needs %lld doubles of scratch for %lld nodes and %lld walkers; "
                "it holds %lld (64 + 6 per 4096 walkers + 12 per 4096 nodes must fit)",
                (long long)need, (long long)N, (long long)nw, (long long)rwmi::kNoAllocDoubles);
  HIPCHK(d, hipSetDevice(d->device));
  double* sc = nullptr;
  HIPCHK(d, rwmi::noalloc_scratch(&sc));
  double* outd = sc;
  double* refd = sc + 32;
  double* pw = sc + 64;
  double* pn = pw + 6 * nbw;
  HIPCHK(d, hipMemcpyAsync(refd, d->ref, 24, hipMemcpyHostToDevice, d->stream));
  HIPCHK(d, rwmi::launch_moments(d->prec, d->dv, 0, N, nw, refd, pw, pn, outd, d->stream));
  double h[32];
  HIPCHK(d, hipMemcpyAsync(h, outd, sizeof h, hipMemcpyDeviceToHost, d->stream));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  fill_moments(d, h, out);
  return RWMI_OK;
}

rwmi_status rwmi_debug_set(rwmi_domain* d, int32_t key, int64_t value) {
  if (!d) return fail(d, RWMI_EINVAL, "null domain");
  HIPCHK(d, hipSetDevice(d->device));
  switch (key) {
    case RWMI_KEY_MAX_BISECT:
      if (value < 1 || value > 100000) return fail(d, RWMI_EINVAL, "max_bisect out of range");
      d->hv.max_bisect = (int32_t)value;
      drop_graph(d);
      if (d->batch) d->batch->dirty = true;
      return upload_view(d);
    case RWMI_KEY_USE_GRAPH:
      d->use_graph = value != 0;
      if (!d->use_graph) drop_graph(d);
      return RWMI_OK;
    case RWMI_KEY_BLOCK:
      if (value != 128 && value != 256 && value != 512) return fail(d, RWMI_EINVAL, "block must be 128, 256 or 512");
      if ((d->dem || d->hv.ibb) && value != 256)
        return fail(d, RWMI_EINVAL, "domains with coupled particles or bounce-back coupling step with 256 threads");
      d->bs = (int)value;
      drop_graph(d);
      // a batch holding it regroups it (if the batch launches members with
      // their own block sizes); its own work map serves steps on its own
      if (d->batch) d->batch->dirty = true;
      return upload_workmaps(d);
    case RWMI_KEY_TIMING:
      if (value < 0 || value > (1 << 20)) return fail(d, RWMI_EINVAL, "timing period out of range");
      d->timing = value != 0;
      d->timing_every = value > 0 ? (uint32_t)value : 1u;
      return RWMI_OK;
    case RWMI_KEY_STEP_FLAGS:
      if (value < 0 || value > 3) return fail(d, RWMI_EINVAL, "step flags must be in 0..3");
      d->flags = (int)value;
      drop_graph(d);
      return RWMI_OK;
    case RWMI_KEY_STREAMING: {
      if (value != 1 && value != 2) return fail(d, RWMI_EINVAL, "streaming must be 1 (two lattices) or 2 (in place)");
      if (d->stepped || d->batch) return fail(d, RWMI_ESTATE, "the streaming layout is chosen before the first step");
      const int ip = value == 2 ? 1 : 0;
      if (ip && d->hv.ibb) return fail(d, RWMI_EINVAL, "bounce-back coupling streams between two lattices");
      if (ip == d->hv.inplace) return RWMI_OK;
      if (!ip && !d->hv.fB) {
        void* fB;
        rwmi_status st;
        if ((st = alloc_into(d, fB, rwmi::f_elems(d->hv.N) * elem_size(d->prec))) != RWMI_OK) return st;
        d->hv.fB = fB;
      }
      d->hv.inplace = ip;
      drop_graph(d);
      if (upload_view(d) != RWMI_OK) return RWMI_EDEVICE;
      HIPCHK(d, rwmi::launch_init(d->prec, d->dv, 0, d->hv.N, d->desc.u0, d->stream));
      HIPCHK(d, hipStreamSynchronize(d->stream));
      return RWMI_OK;
    }
    case RWMI_KEY_SORT_EVERY:
      if (value < 0 || value > (1 << 20)) return fail(d, RWMI_EINVAL, "sort interval out of range");
      d->sort_every = (int)value;
      drop_graph(d);
      if (d->batch) d->batch->dirty = true;
      return RWMI_OK;
    default:
      return fail(d, RWMI_EINVAL, "unknown key %d", key);
  }
}

rwmi_status rwmi_read_kernel_times(rwmi_domain* d, double* ms, uint64_t* launches, uint64_t* fluid_steps,
                                   uint64_t* walker_steps) {
  if (!d || !ms || !launches || !fluid_steps || !walker_steps) return fail(d, RWMI_EINVAL, "null argument");
  HIPCHK(d, hipSetDevice(d->device));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  *ms = 0.0;
  *launches = 0;
  *fluid_steps = 0;
  *walker_steps = 0;
  for (auto& r : d->evrec) {
    float t = 0.0f;
    HIPCHK(d, hipEventElapsedTime(&t, d->evpool[r.ev], d->evpool[r.ev + 1]));
    *ms += t;
    *launches += r.launches;
    *fluid_steps += r.fluid;
    *walker_steps += r.walkers;
  }
  d->evrec.clear();
  if (d->evdem.empty()) d->evused = 0;
  return RWMI_OK;
}

rwmi_status rwmi_read_coupling_times(rwmi_domain* d, double* ms_update, uint64_t* n_update, double* ms_prologue,
                                     uint64_t* n_prologue) {
  if (!d || !ms_update || !n_update || !ms_prologue || !n_prologue) return fail(d, RWMI_EINVAL, "null argument");
  HIPCHK(d, hipSetDevice(d->device));
  HIPCHK(d, hipStreamSynchronize(d->stream));
  *ms_update = *ms_prologue = 0.0;
  *n_update = *n_prologue = 0;
  for (auto& r : d->evdem) {
    float t = 0.0f;
    HIPCHK(d, hipEventElapsedTime(&t, d->evpool[r.first], d->evpool[r.first + 1]));
    if (r.second == 1) {
      *ms_update += t;
      *n_update += 1;
    } else {
      *ms_prologue += t;
      *n_prologue += 1;
    }
  }
  d->evdem.clear();
  if (d->evrec.empty()) d->evused = 0;
  return RWMI_OK;
}

const char* rwmi_last_error(const rwmi_domain* d) { return d ? d->err.c_str() : g_err.c_str(); }

rwmi_status rwmi_device_normals(int32_t device, uint64_t seed, uint32_t t, uint32_t purpose, uint64_t n, double* z) {
  if (!z && n) return fail(nullptr, RWMI_EINVAL, "null output");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, RWMI_EDEVICE, "hipSetDevice failed");
  if (n == 0) return RWMI_OK;
  double* dz = nullptr;
  if (hipMalloc(&dz, 24 * n) != hipSuccess) return fail(nullptr, RWMI_ENOMEM, "hipMalloc failed");
  hipError_t e = rwmi::launch_normals(seed, t, purpose, (int64_t)n, dz, nullptr);
  if (e == hipSuccess) e = hipMemcpy(z, dz, 24 * n, hipMemcpyDeviceToHost);
  (void)hipFree(dz);
  if (e != hipSuccess) return fail(nullptr, RWMI_EDEVICE, "normals: %s", hipGetErrorString(e));
  return RWMI_OK;
}

rwmi_status rwmi_stream_probe(int32_t streams, int32_t elem_bytes, int32_t tiled, uint64_t n, const void* src,
                              void* dst, void* stream) {
  if (!src || !dst) return fail(nullptr, RWMI_EINVAL, "null buffer");
  if (!(streams == 1 || streams == 2 || streams == 4 || streams == 8 || streams == 19))
    return fail(nullptr, RWMI_EINVAL, "streams must be 1, 2, 4, 8 or 19");
  if (elem_bytes != 4 && elem_bytes != 2) return fail(nullptr, RWMI_EINVAL, "elem_bytes must be 4 or 2");
  if (n == 0 || n % 256 != 0 || n >= (1ull << 32)) return fail(nullptr, RWMI_EINVAL, "n must be a positive multiple of 256 below 2^32");
  const hipError_t e = rwmi::launch_stream_probe(streams, elem_bytes, tiled != 0, n, src, dst, (hipStream_t)stream);
  if (e != hipSuccess) return fail(nullptr, RWMI_EDEVICE, "stream probe: %s", hipGetErrorString(e));
  return RWMI_OK;
}

rwmi_status rwmi_dispersion_fit(const double* t, const double* sigma2, uint32_t n, uint32_t i0, double two_r,
                                double u_slip, double phi, double* K, double* D_alpha, double* offset) {
  if (!t || !sigma2 || !K || !D_alpha) return fail(nullptr, RWMI_EINVAL, "null argument");
  if (n < i0 + 2) return fail(nullptr, RWMI_EINVAL, "need at least two samples");
  if (u_slip == 0.0 || !(phi < 1.0) || two_r == 0.0) return fail(nullptr, RWMI_EINVAL, "u_slip, phi or 2R invalid");
  // centred least squares (two passes) for numerical stability
  const double m = (double)(n - i0);
  double st = 0.0, ss = 0.0;
  for (uint32_t i = i0; i < n; ++i) {
    st += t[i];
    ss += sigma2[i] / (two_r * two_r);
  }
  const double tb = st / m, sb = ss / m;
  double sxy = 0.0, sxx = 0.0;
  for (uint32_t i = i0; i < n; ++i) {
    const double dt = t[i] - tb;
    sxy += dt * (sigma2[i] / (two_r * two_r) - sb);
    sxx += dt * dt;
  }
  if (sxx == 0.0) return fail(nullptr, RWMI_EINVAL, "all sample times equal");
  const double b = sxy / sxx;
  *K = b * two_r / u_slip;
  *D_alpha = *K / (1.0 - phi);
  if (offset) *offset = sb - b * tb;
  return RWMI_OK;
}

rwmi_status rwmi_dispersion_from_moments(const rwmi_moments* ser, uint32_t n, uint32_t i0, int32_t disp_axis,
                                         int32_t flow_axis, uint64_t n_nodes, double two_r, double* sigma2,
                                         rwmi_dispersion* out) {
  if (!ser || !out) return fail(nullptr, RWMI_EINVAL, "null argument");
  if (disp_axis < 0 || disp_axis > 2 || flow_axis < 0 || flow_axis > 2) return fail(nullptr, RWMI_EINVAL, "axis out of range");
  if (n_nodes == 0) return fail(nullptr, RWMI_EINVAL, "n_nodes must be > 0");
  if (n < i0 + 2) return fail(nullptr, RWMI_EINVAL, "need at least two samples in the fit");
  std::vector<double> t(n), s2(n);
  double umax = -INFINITY, vmax = -INFINITY, solid = 0.0;
  uint32_t nsolid = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const rwmi_moments& m = ser[i];
    if (m.n_walkers == 0) return fail(nullptr, RWMI_EINVAL, "sample %u has no walkers", i);
    const double N = (double)m.n_walkers;
    const double mean = m.sum[disp_axis] / N;
    t[i] = (double)m.step;
    s2[i] = m.sumsq[disp_axis] / N - mean * mean;
    if (m.fluid_u[flow_axis] > umax) umax = m.fluid_u[flow_axis];
    if (m.particle_v[flow_axis] > vmax) vmax = m.particle_v[flow_axis];
    if (m.step > 0) {
      solid += m.solid_volume;
      nsolid += 1;
    }
  }
  if (sigma2) std::memcpy(sigma2, s2.data(), sizeof(double) * n);
  out->u_slip = std::fabs(umax - vmax);
  out->phi = nsolid ? (solid / (double)nsolid) / (double)n_nodes : 0.0;
  return rwmi_dispersion_fit(t.data(), s2.data(), n, i0, two_r, out->u_slip, out->phi, &out->K, &out->D_alpha,
                             &out->offset);
}

// Least-squares Gaussian through (x_k, y_k) (the concentration-profile fit
// of Sec. 4): Levenberg-Marquardt on (A, mu, s2), started from the weighted
// moments of the profile.
static double gauss_sse(const double* x, const double* y, uint32_t n, const double p[3]) {
  double s = 0.0;
  for (uint32_t k = 0; k < n; ++k) {
    const double d = x[k] - p[1];
    const double r = y[k] - p[0] * std::exp(-0.5 * d * d / p[2]);
    s += r * r;
  }
  return s;
}

// Solve the 3x3 system A z = b by Gaussian elimination with partial pivoting.
static bool solve3(double A[3][3], double b[3], double z[3]) {
  int idx[3] = {0, 1, 2};
  for (int c = 0; c < 3; ++c) {
    int piv = c;
    for (int r = c + 1; r < 3; ++r)
      if (std::fabs(A[idx[r]][c]) > std::fabs(A[idx[piv]][c])) piv = r;
    std::swap(idx[c], idx[piv]);
    const double a = A[idx[c]][c];
    if (a == 0.0 || !std::isfinite(a)) return false;
    for (int r = c + 1; r < 3; ++r) {
      const double f = A[idx[r]][c] / a;
      for (int k = c; k < 3; ++k) A[idx[r]][k] -= f * A[idx[c]][k];
      b[idx[r]] -= f * b[idx[c]];
    }
  }
  for (int c = 2; c >= 0; --c) {
    double v = b[idx[c]];
    for (int k = c + 1; k < 3; ++k) v -= A[idx[c]][k] * z[k];
    z[c] = v / A[idx[c]][c];
  }
  return true;
}

rwmi_status rwmi_gaussian_fit(const double* x, const double* y, uint32_t n, double* amp, double* mean, double* var) {
  if (!x || !y || !amp || !mean || !var) return fail(nullptr, RWMI_EINVAL, "null argument");
  if (n < 3) return fail(nullptr, RWMI_EINVAL, "a Gaussian fit needs at least three points");
  double w = 0.0, m1 = 0.0, top = 0.0;
  uint32_t npos = 0;
  for (uint32_t k = 0; k < n; ++k) {
    if (y[k] > 0.0) {
      w += y[k];
      m1 += y[k] * x[k];
      ++npos;
    }
    top = std::max(top, y[k]);
  }
  if (npos < 3) return fail(nullptr, RWMI_EINVAL, "a Gaussian fit needs at least three positive values");
  double p[3] = {top, m1 / w, 0.0};
  for (uint32_t k = 0; k < n; ++k)
    if (y[k] > 0.0) p[2] += y[k] * (x[k] - p[1]) * (x[k] - p[1]);
  p[2] = p[2] > 0.0 ? p[2] / w : 1.0;
  double sse = gauss_sse(x, y, n, p), lam = 1e-3;
  for (int it = 0; it < 500; ++it) {
    double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, g[3] = {0, 0, 0};
    for (uint32_t k = 0; k < n; ++k) {
      const double d = x[k] - p[1];
      const double e = std::exp(-0.5 * d * d / p[2]);
      const double J[3] = {e, p[0] * e * d / p[2], 0.5 * p[0] * e * d * d / (p[2] * p[2])};
      const double r = y[k] - p[0] * e;
      for (int a = 0; a < 3; ++a) {
        g[a] += J[a] * r;
        for (int b = 0; b < 3; ++b) H[a][b] += J[a] * J[b];
      }
    }
    bool improved = false;
    double q[3] = {0, 0, 0}, sq = sse;
    for (int tries = 0; tries < 40 && !improved; ++tries) {
      double A[3][3], bb[3] = {g[0], g[1], g[2]}, z[3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] = H[a][b] + (a == b ? lam * H[a][a] : 0.0);
      if (!solve3(A, bb, z)) {
        lam *= 10.0;
        continue;
      }
      for (int a = 0; a < 3; ++a) q[a] = p[a] + z[a];
      if (q[2] > 0.0 && (sq = gauss_sse(x, y, n, q)) <= sse) improved = true;
      else lam *= 10.0;
    }
    if (!improved) break;
    double change = 0.0;
    for (int a = 0; a < 3; ++a) {
      change = std::max(change, std::fabs(q[a] - p[a]) / std::max(std::fabs(q[a]), 1e-300));
      p[a] = q[a];
    }
    sse = sq;
    lam = std::max(lam * 0.1, 1e-12);
    if (change < 1e-14) break;
  }
  *amp = p[0];
  *mean = p[1];
  *var = p[2];
  return RWMI_OK;
}

// ---------------------------------------------------------------- batch

static rwmi_status bfail(rwmi_batch* b, rwmi_status st, const char* msg) {
  if (b) b->err = msg;
  g_err = msg;
  return st;
}

rwmi_status rwmi_batch_create(int32_t device, void* stream, rwmi_batch** out) {
  if (!out) return bfail(nullptr, RWMI_EINVAL, "null argument");
  if (hipSetDevice(device) != hipSuccess) return bfail(nullptr, RWMI_EDEVICE, "hipSetDevice failed");
  rwmi_batch* b = new rwmi_batch();
  b->device = device;
  if (stream) {
    b->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return bfail(nullptr, RWMI_EDEVICE, "hipStreamCreate failed");
    }
    b->own_stream = true;
  }
  *out = b;
  return RWMI_OK;
}

static void batch_drop_graph(rwmi_batch* b) {
  if (b->gexec) {
    // no launch of the executable graph may still be in flight
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->gsteps = 0;
  }
}

static void batch_free_groups(rwmi_batch* b) {
  for (void* p : b->owned) (void)hipFree(p);
  b->owned.clear();
  b->groups.clear();
}

rwmi_status rwmi_batch_add(rwmi_batch* b, rwmi_domain* d) {
  if (!b || !d) return bfail(b, RWMI_EINVAL, "null argument");
  if (d->batch) return bfail(b, RWMI_ESTATE, "domain already in a batch");
  if (d->device != b->device) return bfail(b, RWMI_EINVAL, "domain lives on another device");
  if (hipSetDevice(d->device) != hipSuccess) return bfail(b, RWMI_EDEVICE, "hipSetDevice failed");
  if (d->dem || d->hv.ibb)
    return bfail(b, RWMI_EINVAL, "domains with coupled particles or bounce-back coupling are stepped alone");
  if (finalize_particles(d) != RWMI_OK) return bfail(b, RWMI_EDEVICE, d->err.c_str());
  d->batch = b;
  b->members.push_back(d);
  b->dirty = true;
  return RWMI_OK;
}

rwmi_status rwmi_batch_remove(rwmi_batch* b, rwmi_domain* d) {
  if (!b || !d) return bfail(b, RWMI_EINVAL, "null argument");
  auto it = std::find(b->members.begin(), b->members.end(), d);
  if (it == b->members.end()) return bfail(b, RWMI_EINVAL, "domain not in this batch");
  if (hipSetDevice(b->device) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess)
    return bfail(b, RWMI_EDEVICE, "batch synchronisation failed");
  b->members.erase(it);
  d->batch = nullptr;
  b->dirty = true;
  return RWMI_OK;
}

// Rebuild the per-precision view arrays and block maps of the batch.
static rwmi_status batch_rebuild(rwmi_batch* b) {
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, RWMI_EDEVICE, "batch sync failed");
  batch_drop_graph(b);
  batch_free_groups(b);
  static const int kBlockSizes[3] = {128, 256, 512};
  for (int key = 0; key < 24; ++key) {
    const int prec = key >> 3, ip = (key >> 2) & 1, bsi = key & 3;
    if (bsi > 2) continue;
    const int gbs = kBlockSizes[bsi];
    rwmi_batch::Group g;
    g.prec = prec;
    g.inplace = ip;
    g.bs = gbs;
    for (rwmi_domain* d : b->members)
      if (d->prec == prec && d->hv.inplace == ip && (b->member_blocks ? d->bs : b->bs) == gbs) g.doms.push_back(d);
    if (g.doms.empty()) continue;
    const int nd = (int)g.doms.size();
    std::vector<DomView> hv(nd);
    std::vector<int32_t> boff(kRoles * (nd + 1));
    int64_t acc[kRoles] = {0, 0, 0};
    for (int i = 0; i < nd; ++i) {
      int bl[kRoles];
      role_blocks(g.doms[i], gbs, bl);
      for (int k = 0; k < kRoles; ++k) {
        boff[k * (nd + 1) + i] = (int32_t)acc[k];
        acc[k] += bl[k];
      }
      hv[i] = g.doms[i]->hv;
    }
    for (int k = 0; k < kRoles; ++k) {
      if (acc[k] > (int64_t)1 << 28) return bfail(b, RWMI_EINVAL, "batch too large for one launch");
      boff[k * (nd + 1) + nd] = (int32_t)acc[k];
      g.blocks[k] = (int)acc[k];
    }
    if (hipMalloc(&g.views, sizeof(DomView) * nd) != hipSuccess ||
        hipMalloc(&g.boff, sizeof(int32_t) * boff.size()) != hipSuccess)
      return bfail(b, RWMI_ENOMEM, "batch allocation failed");
    b->owned.push_back(g.views);
    b->owned.push_back(g.boff);
    if (hipMemcpy(g.views, hv.data(), sizeof(DomView) * nd, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g.boff, boff.data(), sizeof(int32_t) * boff.size(), hipMemcpyHostToDevice) != hipSuccess)
      return bfail(b, RWMI_EDEVICE, "batch upload failed");
    b->groups.push_back(g);
  }
  b->dirty = false;
  return RWMI_OK;
}

// A launch group of n steps for every member: per precision group the same
// launches as a single domain (prologue-only launch, then n + 1 fused
// launches), each over all members of the group, then the step counters
// advance by n.
static rwmi_status batch_enqueue_group(rwmi_batch* b, uint32_t n, bool capturing) {
  hipStream_t A = b->stream;
  for (int j = -1; j <= (int)n; ++j) {
    for (auto& g : b->groups)
      for (size_t i = 0; i < g.doms.size() && j >= 0; ++i) {
        rwmi_domain* d = g.doms[i];
        if (!sort_before(d, (uint32_t)j, n, capturing)) continue;
        if (rwmi::launch_sort(g.prec, g.views, (int)i, d->hv.nw, d->sort, A) != hipSuccess)
          return bfail(b, RWMI_EDEVICE, "batch sort failed");
        if (!capturing) d->sorted_at = d->steps + (uint32_t)j;
      }
    for (auto& g : b->groups) {
      rwmi::StepArgs a{};
      a.views = g.views;
      a.boff = g.boff;
      a.nd = (int)g.doms.size();
      launch_roles(g.blocks, j, n, a.nb);
      a.flags = b->flags | (j == (int)n - 1 ? rwmi::kFlagDensity : 0);
      a.inplace = g.inplace;
      a.j = j;
      if (a.nb[0] + a.nb[1] + a.nb[2] == 0) continue;
      if (rwmi::launch_step(g.prec, g.bs, a, A) != hipSuccess) return bfail(b, RWMI_EDEVICE, "batch launch failed");
    }
  }
  for (auto& g : b->groups)
    if (rwmi::launch_advance(g.views, (int)g.doms.size(), n, A) != hipSuccess)
      return bfail(b, RWMI_EDEVICE, "batch advance failed");
  return RWMI_OK;
}

rwmi_status rwmi_batch_step(rwmi_batch* b, uint32_t n_steps) {
  if (!b) return bfail(b, RWMI_EINVAL, "null batch");
  if (hipSetDevice(b->device) != hipSuccess) return bfail(b, RWMI_EDEVICE, "hipSetDevice failed");
  for (rwmi_domain* d : b->members)
    if (d->stream != b->stream && hipStreamSynchronize(d->stream) != hipSuccess)
      return bfail(b, RWMI_EDEVICE, "member synchronisation failed");
  if (b->dirty) {
    rwmi_status st = batch_rebuild(b);
    if (st != RWMI_OK) return st;
  }
  if (b->members.empty()) return RWMI_OK;
  uint32_t left = n_steps;
  if (b->use_graph && n_steps >= 2) {
    const uint32_t k = std::min<uint32_t>(n_steps, kGraphSteps);
    if (!b->gexec || b->gsteps != k) {
      batch_drop_graph(b);
      hipGraph_t g;
      if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bfail(b, RWMI_EDEVICE, "capture failed");
      if (batch_enqueue_group(b, k, true) != RWMI_OK) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(b->stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        return RWMI_EDEVICE;
      }
      if (hipStreamEndCapture(b->stream, &g) != hipSuccess) return bfail(b, RWMI_EDEVICE, "end capture failed");
      hipError_t e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return bfail(b, RWMI_EDEVICE, "graph instantiate failed");
      b->gsteps = k;
    }
    while (left >= b->gsteps) {
      if (hipGraphLaunch(b->gexec, b->stream) != hipSuccess) return bfail(b, RWMI_EDEVICE, "graph launch failed");
      left -= b->gsteps;
      for (rwmi_domain* d : b->members) {
        if (d->sort_every > 0 && d->hv.nw > 0) d->sorted_at = d->steps;  // every replay sorts at its start
        d->steps += b->gsteps;
      }
    }
  }
  if (left > 0) {
    rwmi_status st = batch_enqueue_group(b, left, false);
    if (st != RWMI_OK) return st;
    for (rwmi_domain* d : b->members) d->steps += left;
  }
  for (rwmi_domain* d : b->members) d->stepped = true;
  // member reads run on the members' streams: order them after this work
  hipEvent_t ev;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
    (void)hipEventRecord(ev, b->stream);
    for (rwmi_domain* d : b->members)
      if (d->stream != b->stream) (void)hipStreamWaitEvent(d->stream, ev, 0);
    (void)hipEventDestroy(ev);
  }
  return RWMI_OK;
}

rwmi_status rwmi_batch_set(rwmi_batch* b, int32_t key, int64_t value) {
  if (!b) return bfail(b, RWMI_EINVAL, "null batch");
  switch (key) {
    case RWMI_KEY_USE_GRAPH:
      b->use_graph = value != 0;
      if (!b->use_graph) batch_drop_graph(b);
      return RWMI_OK;
    case RWMI_KEY_BLOCK:
      if (value != 128 && value != 256 && value != 512) return bfail(b, RWMI_EINVAL, "block must be 128, 256 or 512");
      b->bs = (int)value;
      b->dirty = true;
      return RWMI_OK;
    case RWMI_KEY_STEP_FLAGS:
      if (value < 0 || value > 3) return bfail(b, RWMI_EINVAL, "step flags must be in 0..3");
      b->flags = (int)value;
      batch_drop_graph(b);
      return RWMI_OK;
    case RWMI_KEY_MEMBER_BLOCKS:
      if (value != 0 && value != 1) return bfail(b, RWMI_EINVAL, "member blocks must be 0 or 1");
      b->member_blocks = value != 0;
      b->dirty = true;
      return RWMI_OK;
    default:
      return bfail(b, RWMI_EINVAL, "unknown batch key");
  }
}

rwmi_status rwmi_batch_synchronize(rwmi_batch* b) {
  if (!b) return bfail(b, RWMI_EINVAL, "null batch");
  if (hipSetDevice(b->device) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess)
    return bfail(b, RWMI_EDEVICE, "batch synchronisation failed");
  return RWMI_OK;
}

void rwmi_batch_destroy(rwmi_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  for (rwmi_domain* d : b->members) d->batch = nullptr;
  batch_drop_graph(b);
  batch_free_groups(b);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
