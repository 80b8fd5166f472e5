// V-pass, streaming part (FP32), one work-group per tile: W = (M_i - S_i)^T U_i
// over row splits.
#include "rpca_vpass_kernel.h"

namespace rpca {

template <int RT, int NS>
static hipError_t launch_vpass_t(const DevParams& p, int mode, const float* U, int64_t u_stride,
                                 const float* Uold, const float* Vold, double* fin_Ginv,
                                 hipStream_t st) {
  const int fin = fin_Ginv ? 1 : 0;
  dim3 grid(p.ng64 * p.vsplit + (fin ? 2 : 0)), block(256);
  auto go = [&](auto kg) {
    constexpr int KG = decltype(kg)::value;
    if (mode == kSZero)
      hipLaunchKernelGGL((k_vpass<RT, NS, kSZero, KG, false>), grid, block, 0, st, p, U, u_stride,
                         Uold, Vold, fin_Ginv, fin);
    else if (mode == kSStored)
      hipLaunchKernelGGL((k_vpass<RT, NS, kSStored, KG, false>), grid, block, 0, st, p, U,
                         u_stride, Uold, Vold, fin_Ginv, fin);
    else
      hipLaunchKernelGGL((k_vpass<RT, NS, kSRecompute, KG, false>), grid, block, 0, st, p, U,
                         u_stride, Uold, Vold, fin_Ginv, fin);
  };
  if (p.vcols == 4)
    go(std::integral_constant<int, 4>{});
  else
    go(std::integral_constant<int, 1>{});
  return hipGetLastError();
}

// The first round (S = 0) always runs one work-group per tile.
hipError_t launch_vpass(const DevParams& p, int mode, const float* U, int64_t u_stride,
                        const float* Uold, const float* Vold, double* fin_Ginv, hipStream_t st) {
  if (p.RP > kFoldMaxRP)
    return fin_Ginv ? hipErrorInvalidValue : launch_vpass_wide(p, mode, U, u_stride, Uold, Vold, st);
  if (mode == kSSparse) return launch_vpass_sparse(p, U, u_stride, fin_Ginv, st);
  if (p.vqueue && mode != kSZero)
    return launch_vpass_queue(p, mode, U, u_stride, Uold, Vold, fin_Ginv, st);
  return with_rank(p, [&](auto rt, auto ns) {
    return launch_vpass_t<decltype(rt)::value, decltype(ns)::value>(p, mode, U, u_stride, Uold,
                                                                   Vold, fin_Ginv, st);
  });
}

}  // namespace rpca
