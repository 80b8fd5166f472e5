// S-pass (FP32), one work-group per tile: fused U V_i^T, soft-threshold,
// Lambda V_i and the U-step terms.
#include "rpca_spass_kernel.h"

namespace rpca {

template <int RT, int NS>
static hipError_t launch_spass_t(const DevParams& p, const float* U, int64_t u_stride, float* Sout,
                                 int64_t lds_out, int emit_only, int client_base,
                                 int client_count, hipStream_t st) {
  // Stored-S rounds and the rebuilt-S ones take the same column phases, so
  // both sum P in the same order.
  const dim3 grid(p.nrb, client_count);
  if (p.sphases == 1) {
    if (Sout)
      hipLaunchKernelGGL((k_spass<RT, NS, kSOutDense, 1, false>), grid, dim3(256), 0, st, p, U, u_stride,
                         Sout, lds_out, emit_only, client_base);
    else
      hipLaunchKernelGGL((k_spass<RT, NS, kSOutNone, 1, false>), grid, dim3(256), 0, st, p, U,
                         u_stride, Sout, lds_out, emit_only, client_base);
  } else {
    if (Sout)
      hipLaunchKernelGGL((k_spass<RT, NS, kSOutDense, 2, false>), grid, dim3(512), 0, st, p, U, u_stride,
                         Sout, lds_out, emit_only, client_base);
    else
      hipLaunchKernelGGL((k_spass<RT, NS, kSOutNone, 2, false>), grid, dim3(512), 0, st, p, U,
                         u_stride, Sout, lds_out, emit_only, client_base);
  }
  return hipGetLastError();
}

// Launches over all clients may run from the tile queue; the S emission of a
// client range always runs one work-group per tile.
hipError_t launch_spass(const DevParams& p, const float* U, int64_t u_stride, float* Sout,
                        int64_t lds_out, int emit_only, int client_base, int client_count,
                        hipStream_t st) {
  if (p.RP > kFoldMaxRP)
    return launch_spass_wide(p, U, u_stride, Sout, lds_out, emit_only, client_base, client_count,
                             st);
  const bool all = !emit_only && client_base == 0 && client_count == p.E;
  if (all && !Sout && p.Smask) return launch_spass_sparse(p, U, u_stride, st);
  if (p.squeue && all) return launch_spass_queue(p, U, u_stride, Sout, lds_out, st);
  return with_rank(p, [&](auto rt, auto ns) {
    return launch_spass_t<decltype(rt)::value, decltype(ns)::value>(
        p, U, u_stride, Sout, lds_out, emit_only, client_base, client_count, st);
  });
}

}  // namespace rpca
