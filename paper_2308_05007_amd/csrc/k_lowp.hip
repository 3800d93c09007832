// FP32 / FP16-storage / BF16-storage kernels (collision and walker
// arithmetic in float; contraction to FMA allowed).
#include "launch.h"
#include "step_impl.h"

namespace rwmi {

template <int P, bool IP>
static void step_bs(int bs, unsigned g, const StepArgs& a, hipStream_t s) {
  switch (bs) {
    case 128: k_step<P, 128, IP><<<g, 128, 0, s>>>(a, a.views, a.boff); break;
    case 512: k_step<P, 512, IP><<<g, 512, 0, s>>>(a, a.views, a.boff); break;
    default: k_step<P, 256, IP><<<g, 256, 0, s>>>(a, a.views, a.boff); break;
  }
}

template <int P>
static void step_layout(int bs, unsigned g, const StepArgs& a, hipStream_t s) {
  if (a.flags & kFlagIbb) {  // bounce-back coupling: two lattices, 256 threads per block; the link
                             // pass carries the coupled particles' momentum exchange
    k_step<P, 256, false, false, true><<<g, 256, 0, s>>>(a, a.views, a.boff);
    return;
  }
  if (a.flags & kFlagDem) {  // coupled particles: 256 threads per block
    if (a.inplace) k_step<P, 256, true, true><<<g, 256, 0, s>>>(a, a.views, a.boff);
    else k_step<P, 256, false, true><<<g, 256, 0, s>>>(a, a.views, a.boff);
    return;
  }
  if (a.inplace) step_bs<P, true>(bs, g, a, s);
  else step_bs<P, false>(bs, g, a, s);
}

hipError_t launch_step_lowp(int prec, int bs, const StepArgs& a, hipStream_t s) {
  const unsigned g = (unsigned)step_grid(a.nb, (a.flags & kFlagXcd) != 0);
  if (g == 0) return hipSuccess;
  if (prec == P32) step_layout<P32>(bs, g, a, s);
  else if (prec == P16) step_layout<P16>(bs, g, a, s);
  else step_layout<PB16>(bs, g, a, s);
  return hipGetLastError();
}

template <int P>
static void links(const DomView* v, int dom, int32_t j, bool dem, unsigned blocks, hipStream_t s) {
  if (dem) k_ibb_links<P, true><<<blocks, 256, 0, s>>>(v, dom, j);
  else k_ibb_links<P, false><<<blocks, 256, 0, s>>>(v, dom, j);
}

hipError_t launch_ibb_links_lowp(int prec, const DomView* v, int dom, int32_t j, bool dem, unsigned blocks,
                                 hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  blocks = kLinkGrid;  // the pass strides over the listed nodes
  if (prec == P32) links<P32>(v, dom, j, dem, blocks, s);
  else if (prec == P16) links<P16>(v, dom, j, dem, blocks, s);
  else links<PB16>(v, dom, j, dem, blocks, s);
  return hipGetLastError();
}

hipError_t launch_init_lowp(int prec, const DomView* v, int dom, int64_t N, const double u0[3], hipStream_t s) {
  const unsigned g = (unsigned)((N + 255) / 256);
  if (prec == P32) k_init<P32><<<g, 256, 0, s>>>(v, dom, u0[0], u0[1], u0[2]);
  else if (prec == P16) k_init<P16><<<g, 256, 0, s>>>(v, dom, u0[0], u0[1], u0[2]);
  else k_init<PB16><<<g, 256, 0, s>>>(v, dom, u0[0], u0[1], u0[2]);
  return hipGetLastError();
}

hipError_t launch_read_f_lowp(int prec, const DomView* v, int dom, int64_t N, double* out, hipStream_t s) {
  const unsigned g = (unsigned)((N + 255) / 256);
  if (prec == P32) k_read_f<P32><<<g, 256, 0, s>>>(v, dom, out);
  else if (prec == P16) k_read_f<P16><<<g, 256, 0, s>>>(v, dom, out);
  else k_read_f<PB16><<<g, 256, 0, s>>>(v, dom, out);
  return hipGetLastError();
}

}  // namespace rwmi
