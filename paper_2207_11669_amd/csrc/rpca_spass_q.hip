// S-pass (FP32), persistent launches over the tile queue.
#include "rpca_spass_kernel.h"

namespace rpca {

template <int RT, int NS>
static hipError_t launch_spass_q_t(const DevParams& p, const float* U, int64_t u_stride,
                                   float* Sout, int64_t lds_out, hipStream_t st) {
  const int ntiles = p.nrb * p.E;
  auto launch = [&](auto kernel, int block) {
    const int groups = pass_groups(kernel, block, ntiles, 1);
    hipLaunchKernelGGL(kernel, dim3(groups), dim3(block), 0, st, p, U, u_stride, Sout, lds_out, 0,
                       0);
  };
  if (p.sphases == 1) {
    if (Sout)
      launch(k_spass<RT, NS, kSOutDense, 1, true>, 256);
    else
      launch(k_spass<RT, NS, kSOutNone, 1, true>, 256);
  } else {
    if (Sout)
      launch(k_spass<RT, NS, kSOutDense, 2, true>, 512);
    else
      launch(k_spass<RT, NS, kSOutNone, 2, true>, 512);
  }
  return hipGetLastError();
}

hipError_t launch_spass_queue(const DevParams& p, const float* U, int64_t u_stride, float* Sout,
                              int64_t lds_out, hipStream_t st) {
  return with_rank(p, [&](auto rt, auto ns) {
    return launch_spass_q_t<decltype(rt)::value, decltype(ns)::value>(p, U, u_stride, Sout,
                                                                     lds_out, st);
  });
}

}  // namespace rpca
