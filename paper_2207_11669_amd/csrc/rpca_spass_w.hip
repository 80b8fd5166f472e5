// S-pass (FP32) at ranks above 64 (five to eight 16-rank tiles, NS = 4 RT:
// the padding ranks are zero in every factor and add exact zeros). One column
// phase (256 threads): the epilogue's P and A_i tiles take up to 141 KB of
// LDS at r = 128, one work-group per compute unit. Every launch form and S
// output, as for the narrower ranks.
#include "rpca_spass_kernel.h"

namespace rpca {

template <int RT>
static hipError_t launch_spass_w_t(const DevParams& p, const float* U, int64_t u_stride,
                                   float* Sout, int64_t lds_out, int emit_only, int client_base,
                                   int client_count, hipStream_t st) {
  constexpr int NS = 4 * RT;
  const bool all = !emit_only && client_base == 0 && client_count == p.E;
  const int ntiles = p.nrb * p.E;
  auto tiles = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(p.nrb, client_count), dim3(256), 0, st, p, U, u_stride, Sout,
                       lds_out, emit_only, client_base);
  };
  auto queue = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(pass_groups(kernel, 256, ntiles, 1)), dim3(256), 0, st, p, U,
                       u_stride, Sout, lds_out, 0, 0);
  };
  if (all && !Sout && p.Smask) {
    if (!p.Sval) return hipErrorInvalidValue;
    if (p.squeue)
      queue(k_spass<RT, NS, kSOutSparse, 1, true>);
    else
      tiles(k_spass<RT, NS, kSOutSparse, 1, false>);
  } else if (p.squeue && all) {
    if (Sout)
      queue(k_spass<RT, NS, kSOutDense, 1, true>);
    else
      queue(k_spass<RT, NS, kSOutNone, 1, true>);
  } else {
    if (Sout)
      tiles(k_spass<RT, NS, kSOutDense, 1, false>);
    else
      tiles(k_spass<RT, NS, kSOutNone, 1, false>);
  }
  return hipGetLastError();
}

hipError_t launch_spass_wide(const DevParams& p, const float* U, int64_t u_stride, float* Sout,
                             int64_t lds_out, int emit_only, int client_base, int client_count,
                             hipStream_t st) {
  if (p.sphases != 1 || p.NS != p.RP / 4) return hipErrorInvalidValue;
  switch (p.RP / 16) {
    case 5: return launch_spass_w_t<5>(p, U, u_stride, Sout, lds_out, emit_only, client_base, client_count, st);
    case 6: return launch_spass_w_t<6>(p, U, u_stride, Sout, lds_out, emit_only, client_base, client_count, st);
    case 7: return launch_spass_w_t<7>(p, U, u_stride, Sout, lds_out, emit_only, client_base, client_count, st);
    case 8: return launch_spass_w_t<8>(p, U, u_stride, Sout, lds_out, emit_only, client_base, client_count, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rpca
