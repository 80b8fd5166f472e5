// S-pass (FP32) over all clients writing S in sparse form (support words and
// packed nonzero values per 16 x 16 tile) for the next V-pass; both launch
// forms.
#include "rpca_spass_kernel.h"

namespace rpca {

template <int RT, int NS>
static hipError_t launch_spass_s_t(const DevParams& p, const float* U, int64_t u_stride,
                                   hipStream_t st) {
  const int ntiles = p.nrb * p.E;
  auto launch = [&](auto kernel, int block, bool queue) {
    if (queue)
      hipLaunchKernelGGL(kernel, dim3(pass_groups(kernel, block, ntiles, 1)), dim3(block), 0, st,
                         p, U, u_stride, nullptr, 0, 0, 0);
    else
      hipLaunchKernelGGL(kernel, dim3(p.nrb, p.E), dim3(block), 0, st, p, U, u_stride, nullptr,
                         0, 0, 0);
  };
  if (p.sphases == 1) {
    if (p.squeue)
      launch(k_spass<RT, NS, kSOutSparse, 1, true>, 256, true);
    else
      launch(k_spass<RT, NS, kSOutSparse, 1, false>, 256, false);
  } else {
    if (p.squeue)
      launch(k_spass<RT, NS, kSOutSparse, 2, true>, 512, true);
    else
      launch(k_spass<RT, NS, kSOutSparse, 2, false>, 512, false);
  }
  return hipGetLastError();
}

hipError_t launch_spass_sparse(const DevParams& p, const float* U, int64_t u_stride,
                               hipStream_t st) {
  if (!p.Smask || !p.Sval) return hipErrorInvalidValue;
  return with_rank(p, [&](auto rt, auto ns) {
    return launch_spass_s_t<decltype(rt)::value, decltype(ns)::value>(p, U, u_stride, st);
  });
}

}  // namespace rpca
