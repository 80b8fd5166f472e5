// V-pass, streaming part (FP32), persistent launches over the tile queue.
#include "rpca_vpass_kernel.h"

namespace rpca {

template <int RT, int NS>
static hipError_t launch_vpass_q_t(const DevParams& p, int mode, const float* U, int64_t u_stride,
                                   const float* Uold, const float* Vold, double* fin_Ginv,
                                   hipStream_t st) {
  const int fin = fin_Ginv ? 1 : 0;
  const int ntiles = p.ng64 * p.vsplit;
  auto launch = [&](auto kernel) {
    const int groups = pass_groups(kernel, 256, ntiles, 1);
    hipLaunchKernelGGL(kernel, dim3(groups + (fin ? 2 : 0)), dim3(256), 0, st, p, U, u_stride,
                       Uold, Vold, fin_Ginv, fin);
  };
  auto go = [&](auto kg) {
    constexpr int KG = decltype(kg)::value;
    if (mode == kSStored)
      launch(k_vpass<RT, NS, kSStored, KG, true>);
    else
      launch(k_vpass<RT, NS, kSRecompute, KG, true>);
  };
  if (p.vcols == 4)
    go(std::integral_constant<int, 4>{});
  else
    go(std::integral_constant<int, 1>{});
  return hipGetLastError();
}

hipError_t launch_vpass_queue(const DevParams& p, int mode, const float* U, int64_t u_stride,
                              const float* Uold, const float* Vold, double* fin_Ginv,
                              hipStream_t st) {
  if (mode != kSStored && mode != kSRecompute) return hipErrorInvalidValue;
  return with_rank(p, [&](auto rt, auto ns) {
    return launch_vpass_q_t<decltype(rt)::value, decltype(ns)::value>(p, mode, U, u_stride, Uold,
                                                                     Vold, fin_Ginv, st);
  });
}

}  // namespace rpca
