// FP32 / FP16-storage / BF16-storage kernels (collision and walker
// arithmetic in float; contraction to FMA allowed).
#include "lbm_impl.h"
#include "walk_impl.h"
#include "launch.h"

namespace rwmi {

template <int P>
static void fluid_bs(int bs, const Work& w, hipStream_t s) {
  switch (bs) {
    case 128: k_fluid<P, 128><<<w.blocks, 128, 0, s>>>(w.views, w.boff, w.nd, w.flags, w.k); break;
    case 512: k_fluid<P, 512><<<w.blocks, 512, 0, s>>>(w.views, w.boff, w.nd, w.flags, w.k); break;
    default: k_fluid<P, 256><<<w.blocks, 256, 0, s>>>(w.views, w.boff, w.nd, w.flags, w.k); break;
  }
}

hipError_t launch_fluid_lowp(int prec, int bs, const Work& w, hipStream_t s) {
  if (prec == P32) fluid_bs<P32>(bs, w, s);
  else if (prec == P16) fluid_bs<P16>(bs, w, s);
  else fluid_bs<PB16>(bs, w, s);
  return hipGetLastError();
}

hipError_t launch_walk_lowp(int bs, const Work& w, hipStream_t s) {
  // every low-precision mode keeps walker offsets and the velocity in float
  switch (bs) {
    case 128: k_walk<P32, 128><<<w.blocks, 128, 0, s>>>(w.views, w.boff, w.nd, w.k); break;
    default: k_walk<P32, 256><<<w.blocks, 256, 0, s>>>(w.views, w.boff, w.nd, w.k); break;
  }
  return hipGetLastError();
}

hipError_t launch_walk_slow_lowp(int bs, const Work& w, hipStream_t s) {
  if (bs == 128) k_walk_slow<P32, 128><<<w.blocks, 128, 0, s>>>(w.views, w.boff, w.nd, w.k);
  else k_walk_slow<P32, 256><<<w.blocks, 256, 0, s>>>(w.views, w.boff, w.nd, w.k);
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
