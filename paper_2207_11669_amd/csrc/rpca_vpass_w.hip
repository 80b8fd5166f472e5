// V-pass, streaming part (FP32), at ranks above 64 (five to eight 16-rank
// tiles, NS = 4 RT: the padding ranks are zero in every factor and add exact
// zeros). One 16-column group per wave (the U operands of four groups would
// not fit the registers), every launch form; the previous round's finalize
// runs as its own launch (its r x r FP64 matrix would not share the LDS).
#include "rpca_vpass_kernel.h"

namespace rpca {

template <int RT>
static hipError_t launch_vpass_w_t(const DevParams& p, int mode, const float* U, int64_t u_stride,
                                   const float* Uold, const float* Vold, hipStream_t st) {
  constexpr int NS = 4 * RT;
  const int ntiles = p.ng64 * p.vsplit;
  // The first round (S = 0) always runs one work-group per tile.
  const bool queue = p.vqueue && mode != kSZero;
  auto launch = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(pass_groups(kernel, 256, ntiles, queue ? 1 : 0)), dim3(256), 0,
                       st, p, U, u_stride, Uold, Vold, nullptr, 0);
  };
  switch (mode) {
    case kSZero:
      launch(k_vpass<RT, NS, kSZero, 1, false>);
      break;
    case kSStored:
      if (queue)
        launch(k_vpass<RT, NS, kSStored, 1, true>);
      else
        launch(k_vpass<RT, NS, kSStored, 1, false>);
      break;
    case kSRecompute:
      if (queue)
        launch(k_vpass<RT, NS, kSRecompute, 1, true>);
      else
        launch(k_vpass<RT, NS, kSRecompute, 1, false>);
      break;
    case kSSparse:
      if (!p.Smask || !p.Sval) return hipErrorInvalidValue;
      if (queue)
        launch(k_vpass<RT, NS, kSSparse, 1, true>);
      else
        launch(k_vpass<RT, NS, kSSparse, 1, false>);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vpass_wide(const DevParams& p, int mode, const float* U, int64_t u_stride,
                             const float* Uold, const float* Vold, hipStream_t st) {
  if (p.vcols != 1 || p.NS != p.RP / 4) return hipErrorInvalidValue;
  switch (p.RP / 16) {
    case 5: return launch_vpass_w_t<5>(p, mode, U, u_stride, Uold, Vold, st);
    case 6: return launch_vpass_w_t<6>(p, mode, U, u_stride, Uold, Vold, st);
    case 7: return launch_vpass_w_t<7>(p, mode, U, u_stride, Uold, Vold, st);
    case 8: return launch_vpass_w_t<8>(p, mode, U, u_stride, Uold, Vold, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rpca
