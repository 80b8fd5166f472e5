// V-pass, streaming part (FP32), reading the sparse S of the previous S-pass;
// both launch forms.
#include "rpca_vpass_kernel.h"

namespace rpca {

template <int RT, int NS>
static hipError_t launch_vpass_s_t(const DevParams& p, const float* U, int64_t u_stride,
                                   double* fin_Ginv, hipStream_t st) {
  const int fin = fin_Ginv ? 1 : 0;
  const int ntiles = p.ng64 * p.vsplit;
  auto launch = [&](auto kernel, bool queue) {
    const int groups = queue ? pass_groups(kernel, 256, ntiles, 1) : ntiles;
    hipLaunchKernelGGL(kernel, dim3(groups + (fin ? 2 : 0)), dim3(256), 0, st, p, U, u_stride,
                       nullptr, nullptr, fin_Ginv, fin);
  };
  auto go = [&](auto kg) {
    constexpr int KG = decltype(kg)::value;
    if (p.vqueue)
      launch(k_vpass<RT, NS, kSSparse, KG, true>, true);
    else
      launch(k_vpass<RT, NS, kSSparse, KG, false>, false);
  };
  if (p.vcols == 4)
    go(std::integral_constant<int, 4>{});
  else
    go(std::integral_constant<int, 1>{});
  return hipGetLastError();
}

hipError_t launch_vpass_sparse(const DevParams& p, const float* U, int64_t u_stride,
                               double* fin_Ginv, hipStream_t st) {
  if (!p.Smask || !p.Sval) return hipErrorInvalidValue;
  return with_rank(p, [&](auto rt, auto ns) {
    return launch_vpass_s_t<decltype(rt)::value, decltype(ns)::value>(p, U, u_stride, fin_Ginv, st);
  });
}

}  // namespace rpca
