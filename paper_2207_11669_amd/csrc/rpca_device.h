// Device helpers shared by the DCF-PCA kernel sources (one translation unit
// per kernel family, compiled in parallel).
#pragma once

// DCF-PCA round on one MI355X (gfx950): hand-written HIP kernels.
//
// One local step of Algorithm 1 (Section 2.2) for every client is
//   V-pass   : W_i = (M_i - S_i)^T U_i, then V_i = W_i (U_i^T U_i + rho I)^{-1}
//              (eq. "condition1", Lemma 4 proof), plus partial V_i^T V_i;
//   S-pass   : R = M_i - U_i V_i^T formed 16x16 tile by tile in registers,
//              S_i = sign(R) max(|R| - lambda, 0) (eq. "optS") written,
//              Lambda = R - S_i = clip(R, -lambda, lambda), and
//              P_i = Lambda V_i accumulated (the data term of grad_U L_i,
//              Lemma 2 proof); L = U V^T never reaches memory;
//   U-update : GRAD  U_i - eta (rho n_i/n U_i - P_i)                (eq. "U_local")
//              CLOSED (P_i + U_i V_i^T V_i)(V_i^T V_i + rho n_i/n I)^{-1}
//              and, at the last local step, the mean over clients (eq. "U_agg")
//              together with partial Gram matrices of the new U;
//   finalize : U^T U + rho I and its FP64 inverse (a Gauss-Jordan sweep, which
//              needs no pivoting on an SPD matrix), and the round's FP64
//              statistics.
// With K = 1 and one V/S alternation, S_i is not stored: the next V-pass
// rebuilds it as soft(M_i - U^(t-1) V_i^T) from the previous factors, which
// gives bitwise the S the S-pass computed, so each round streams M twice and
// nothing else of size m x n.
// The rank-r contractions run on the fp32 MFMA (v_mfma_f32_16x16x4f32); the
// r x r algebra and all reductions that feed a convergence test are FP64.
#include "rpca_internal.h"

#include <cmath>
#include <mutex>
#include <type_traits>

namespace rpca {

typedef float f4 __attribute__((ext_vector_type(4)));

// Global-address-space views. Pointers read from device tables (the client
// table) are not known to be global to the compiler, which then emits flat
// memory instructions; those count against both wait counters and serialise
// the prefetch rings below.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const GLOBAL T* gptr(const T* p) {
  return (const GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ GLOBAL T* gptr_w(T* p) {
  return (GLOBAL T*)p;
}

// Constant-address-space view: loads from a wave-uniform address through it
// go through the scalar cache (used only for data an earlier launch wrote).
#define CONSTANT __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const CONSTANT T* cptr(const T* p) {
  return (const CONSTANT T*)p;
}

// Raw buffer loads. A buffer resource holds a base address and a byte range;
// lanes whose offset falls outside the range read 0 instead of memory, and the
// per-lane offset is 32-bit, so addresses need no 64-bit arithmetic per load.
// Only the per-lane voffset takes part in the range check; the scalar soffset
// is used only where every access is in range by construction.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kBufferDword3 = 0x00020000;  // raw (untyped) buffer, gfx9 family
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, kBufferDword3);
}
__device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ f4 bload4(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
// Raw buffer stores; lanes whose offset falls outside the range write nothing.
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, (int)voff, 0, 0);
}
typedef uint32_t u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bstore64(rsrc_t r, uint32_t voff, uint64_t x) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, (int)voff, 0, 0);
}
typedef uint32_t u4s __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void bstore4(rsrc_t r, uint32_t voff, f4 x) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4s, x), r, (int)voff, 0, 0);
}
// Lane-pair exchanges within a quad of lanes (DPP quad permutations): the
// value of lane l ^ 1, or of lane l ^ 2.
__device__ __forceinline__ float quad_xor1(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float quad_xor2(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x4E, 0xF, 0xF, true));
}
// 4 x 4 transpose within each quad of lanes: lane 4 q + e holds x[v] on
// entry and x'[e'] = (lane 4 q + e')'s x[v] with v = its own e on exit (two
// pair-exchange stages: 2 x 2 blocks across lanes l ^ 2, then entries across
// lanes l ^ 1; scalar selects, 16 instructions).
__device__ __forceinline__ f4 quad_transpose(f4 x) {
  const int e = threadIdx.x & 3;
  const bool h = (e & 2) != 0, o = (e & 1) != 0;
  float x0 = x[0], x1 = x[1], x2 = x[2], x3 = x[3];
  const float a0 = quad_xor2(h ? x0 : x2), a1 = quad_xor2(h ? x1 : x3);
  const float y0 = h ? a0 : x0, y1 = h ? a1 : x1, y2 = h ? x2 : a0, y3 = h ? x3 : a1;
  const float b0 = quad_xor1(o ? y0 : y1), b1 = quad_xor1(o ? y2 : y3);
  x0 = o ? b0 : y0;
  x1 = o ? y1 : b0;
  x2 = o ? b1 : y2;
  x3 = o ? y3 : b1;
  return f4{x0, x1, x2, x3};
}
// Tile queue of a persistent launch (a streaming pass whose grid holds only
// as many work-groups as are resident at once). q[0] is the next tile, q[1]
// counts the work-groups that found the queue empty. One lane takes a tile
// with a vector-memory atomic and the work-group reads it from LDS; the
// leading barrier keeps the previous tile's LDS readers ahead of the next
// tile's writers. Every work-group leaves once the count passes ntiles, so
// the launch always drains; the last one to leave resets both counters for
// the next launch (no memset, so the launch can be replayed from a graph).
// Each tile writes only its own slots of the outputs, so which work-group
// takes which tile changes no result.
__device__ __forceinline__ int queue_next(uint32_t* q, int ntiles) {
  __shared__ int s_tile;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = (int)atomicAdd(&q[0], 1u);
    if (t >= ntiles) {
      const uint32_t left = atomicAdd(&q[1], 1u);
      if (left + 1 == gridDim.x * gridDim.y) {
        atomicExch(&q[0], 0u);
        atomicExch(&q[1], 0u);
      }
    }
    s_tile = t;
  }
  __syncthreads();
  return s_tile;
}

// Byte range of a whole factor layout. The parameter checks keep every such
// layout below 2^31 bytes; a larger value would be a broken invariant, and
// the range is then 0 (every load reads 0) rather than a wrapped 32-bit size.
__device__ __forceinline__ uint32_t range32(int64_t bytes) {
  return bytes >= 0 && bytes < ((int64_t)1 << 31) ? (uint32_t)bytes : 0u;
}
// Bytes of a client block from column j0 on (0 past the end), capped to the
// 32-bit range of a buffer resource.
__device__ __forceinline__ uint32_t block_bytes_from(int n, int j0, int64_t ldm) {
  if (j0 >= n) return 0u;
  const int64_t b = (int64_t)(n - j0) * ldm * 4;
  return b > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)b;
}
// Range of a resource over one 16-column chunk: every offset a chunk uses is
// below 64 ldm <= 0xFFFFFF00 bytes (ldm < 2^26), so kOffNone always falls
// outside it and loads at kOffNone return 0.
constexpr uint32_t kChunkRange = 0xFFFFFF00u;
constexpr uint32_t kOffNone = 0xFFFFFF80u;
__device__ __forceinline__ uint32_t chunk_bytes_from(int n, int j0, int64_t ldm) {
  const uint32_t b = block_bytes_from(n, j0, ldm);
  return b > kChunkRange ? kChunkRange : b;
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  // D[i][j] += sum_k A[i][k] B[k][j] over a 16x16x4 tile. Lane l supplies
  // A[l%16][l/16] and B[l/16][l%16]; D[4*(l/16)+v][l%16] lands in element v.
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr int kFinThreads = 256;                             // finalize work-groups
// Lower-triangle entries per finalize thread for ranks up to R.
constexpr int fin_ept(int R) { return (R * (R + 1) / 2 + kFinThreads - 1) / kFinThreads; }
constexpr int kFinEPT = fin_ept(kFoldMaxRP);  // ranks up to 64 (the folded finalize)

// 1/x for x > 0 without the correctly rounded division sequence: the
// hardware reciprocal estimate refined by two Newton steps (each squares the
// relative error), which lands within an ulp or two of 1/x.
__device__ __forceinline__ double recip_pos(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// In-place inverse of an r x r SPD matrix A (row stride ld, in LDS) by a
// Gauss-Jordan sweep without pivoting, run by the whole work-group (EPT *
// blockDim.x >= r (r + 1) / 2): the k-th pivot is a diagonal entry of a Schur
// complement of an SPD matrix, hence positive, and every step updates the
// matrix in parallel (no serial triangular solves). Step k sets
//   A[k][k] <- 1/p,  A[k][j] <- A[k][j] / p,  A[i][k] <- -A[i][k] / p,
//   A[i][j] <- A[i][j] - A[i][k] A[k][j] / p     (p = A[k][k]).
// Throughout the sweep A[j][i] = A[i][j] when i and j are both swept or both
// not, and -A[i][j] otherwise, exactly (the mirrored update multiplies the
// same two factors), so only the lower triangle is updated and the upper one
// is mirrored at the end, where every index is swept. Step k then needs only
// the cross x_t = A[max(t,k)][min(t,k)]: A[k][j] = x_j, and A[i][k] = x_i for
// i >= k, -x_i for i < k. The threads owning the next step's cross publish it
// during this step into a second LDS vector (double-buffered by step parity),
// so each step costs one barrier. Each thread owns up to EPT lower-triangle
// entries, indexed once and held in registers through the sweep (no other
// thread reads or writes them; the LDS carries the cross vector only), then
// written back with the mirror. A pivot that is not positive (non-SPD or NaN
// input) turns the result into NaN, which the round statistics then expose.
// BATCH: a step's cross reads all go out before the pivot's reciprocal (the
// default up to four entries per thread; the standalone kernels at ranks
// above 64 ask for it with nine). Same values either way.
template <int EPT, bool BATCH = (EPT <= 4)>
__device__ void spd_inverse(double* A, int r, int ld) {
  __shared__ double xb[2][kMaxRank];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nl = r * (r + 1) / 2;
  int ei[EPT], ej[EPT];
  double a[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + q * nt;
    int i = -1, j = -1;
    if (e < nl) {
      i = (int)((sqrtf(8.f * (float)e + 1.f) - 1.f) * 0.5f);
      while (i * (i + 1) / 2 > e) --i;
      while ((i + 1) * (i + 2) / 2 <= e) ++i;
      j = e - i * (i + 1) / 2;
    }
    ei[q] = i;
    ej[q] = j;
    a[q] = i >= 0 ? A[i * ld + j] : 0.0;
  }
  if (tid < r) xb[0][tid] = A[tid * ld];
  // Slots q with an entry in some lane of this wave: tid0 + q nt < nl.
  const int tid0 = __builtin_amdgcn_readfirstlane(tid & ~63);
  const int wq = nl > tid0 ? (nl - tid0 + nt - 1) / nt : 0;
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    const int cur = k & 1, nxt = cur ^ 1;
    const double pv = xb[cur][k];
    // A lane's slot without an entry (ei = ej = -1) reads the cross at 0 and
    // never matches a pivot or a publication index, so no per-lane entry test
    // is needed before the write-back; slots past the wave's last entry
    // (wave-uniform) are skipped.
    auto update = [&](int q, double xi, double xj, double pinv) {
      const int i = ei[q], j = ej[q];
      const double ci = i < k ? -xi : xi;
      double v = a[q] - ci * xj * pinv;
      v = j == k ? -xi * pinv : v;
      v = i == k ? (j == k ? pinv : xj * pinv) : v;
      a[q] = v;
      if (i == k + 1) xb[nxt][j] = v;
      if (j == k + 1) xb[nxt][i] = v;
    };
    if constexpr (BATCH) {
      // The step's cross reads go out together, before the pivot's
      // reciprocal; the three cases are then selects. (With many entries per
      // thread in the folded finalize the held reads would cost more
      // registers than the latency they save.)
      double xi[EPT], xj[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        if (q < wq) {
          xi[q] = xb[cur][max(ei[q], 0)];
          xj[q] = xb[cur][max(ej[q], 0)];
        }
      const double pinv = pv > 0.0 ? recip_pos(pv) : NAN;
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        if (q < wq) update(q, xi[q], xj[q], pinv);
    } else {
      const double pinv = pv > 0.0 ? recip_pos(pv) : NAN;
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        if (q < wq) update(q, xb[cur][max(ei[q], 0)], xb[cur][max(ej[q], 0)], pinv);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q)
    if (ei[q] >= 0) {
      A[ei[q] * ld + ej[q]] = a[q];
      if (ei[q] > ej[q]) A[ej[q] * ld + ei[q]] = a[q];
    }
  __syncthreads();
}

__device__ __forceinline__ double eta_of_round(const DevParams& p, int64_t t) {
  if (p.u_mode != 0) return 0.0;
  return p.eta_sched == 1 ? p.eta0 / sqrt((double)t + 1.0) : p.eta0;
}

// Sum of count strided values in FP64, in a fixed order; loads are issued in
// batches of 16 so that a long list of partials costs a few memory latencies.
template <class T>
__device__ __forceinline__ double sum_strided(const T* __restrict__ x, int count,
                                              int64_t stride) {
  double s = 0.0;
  for (int k = 0; k < count; k += 16) {
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = (k + u < count) ? x[(int64_t)(k + u) * stride] : T(0);
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) t += (double)v[u];
    s += t;
  }
  return s;
}

// Per-thread part of sum_{k < count} load(k) over nt threads, thread t
// taking k = t, t + nt, ...; each batch of 16 loads is issued before
// any of them is used, so a long list costs a few memory latencies rather
// than one per element. Fixed order for a fixed block size.
template <class F>
__device__ __forceinline__ double block_strided_sum(int count, F load, int nt) {
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int k0 = tid; k0 < count; k0 += 16 * nt) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + u * nt;
      v[u] = k < count ? load(k) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u];
  }
  return s;
}

// Store element (a, c) of a factor with `rows` rows into its factor block
// (column-major, A-operand packing, B-operand packing; see rpca_internal.h).
__device__ __forceinline__ void fb_store(float* fb, int64_t rows, int RP, int NS, int a, int c,
                                         float v) {
  fb[(int64_t)c * rows + a] = v;
  const int ch = a >> 4, li = a & 15;
  if (c < 4 * NS) {
    const int g = c / NS, s = c - g * NS;
    fb[fb_pa_off(rows, RP) + ((int64_t)ch * NS + s) * 64 + g * 16 + li] = v;
  }
  const int ct = c >> 4, lane = ((li >> 2) << 4) + (c & 15);
  fb[fb_pb_off(rows, RP, NS) + (((int64_t)ch * (RP >> 4) + ct) * 64 + lane) * 4 + (li & 3)] = v;
  const int NQ = nquads(RP, NS), cq = c - (RP - 16);
  if (cq >= 0 && cq < 4 * NQ)
    fb[fb_pq_off(rows, RP, NS) +
       ((((int64_t)ch * NQ + (cq >> 2)) * 4 + (li >> 2)) * 4 + (cq & 3)) * 4 + (li & 3)] = v;
}

// Store element (a, c), c < RP, of a factor with `rows` rows into its BF16
// packings (hA, hP, hB; see rpca_internal.h): hi = v rounded to nearest
// even, then lo = (v - hi) rounded, one packing block further on.
__device__ __forceinline__ void hb_store(uint16_t* hb, int64_t rows, const DevParams& p, int a,
                                         int c, float v) {
  __bf16* h = reinterpret_cast<__bf16*>(hb);
  const __bf16 hi = (__bf16)v;
  const __bf16 lo = (__bf16)(v - (float)hi);
  const int64_t ia = hb_hA(a, c, p.NK), ip = rows * p.RK + hb_hP(a, c, p.NK),
                ib = 2 * rows * p.RK + hb_hB(a, c, p.RP >> 4), lo_off = hb_elems(rows, p.RK, p.RP);
  h[ia] = hi;
  h[ip] = hi;
  h[ib] = hi;
  h[lo_off + ia] = lo;
  h[lo_off + ip] = lo;
  h[lo_off + ib] = lo;
}

// The same layouts written for NR consecutive rows [row0, row0 + NR) at once
// (row0 and NR multiples of 32) by a 256-thread work-group, from an accessor
// x(i, c) for row row0 + i and rank c < RP (0 at ranks past r): every layout's
// span for these rows is contiguous, so threads walk it in order and each
// store instruction covers whole cache lines, where the per-entry stores
// above scatter one dword or one bf16 per line. hb is null when the context
// keeps no BF16 packings. Same values, same places.
template <int RT, int NR, class X>
__device__ __forceinline__ void factor_store_rows(float* fb, uint16_t* hb, int64_t rows,
                                                  const DevParams& p, int row0, X x) {
  constexpr int RP = 16 * RT;
  static_assert(NR % 32 == 0, "whole 32-row chunks");
  const int tid = threadIdx.x, NS = p.NS, NQ = nquads(RP, NS);
  const int ch16 = row0 >> 4, ch32 = row0 >> 5;
  for (int e = tid; e < RP * NR; e += 256) {  // column-major
    const int c = e / NR, i = e - c * NR;
    fb[(int64_t)c * rows + row0 + i] = x(i, c);
  }
  {  // A-operand packing: per 16-row chunk, NS blocks of 64 lanes
    float* d = fb + fb_pa_off(rows, RP) + (int64_t)ch16 * NS * 64;
    for (int e = tid; e < (NR / 16) * NS * 64; e += 256) {
      const int lane = e & 63, s = (e >> 6) % NS, chl = (e >> 6) / NS;
      d[e] = x(16 * chl + (lane & 15), (lane >> 4) * NS + s);
    }
  }
  {  // B-operand packing: per 16-row chunk, RT tiles of 64 lanes x 4
    float* d = fb + fb_pb_off(rows, RP, NS) + (int64_t)ch16 * RT * 256;
    for (int e = tid; e < (NR / 16) * RT * 256; e += 256) {
      const int el = e & 3, lane = (e >> 2) & 63, ct = (e >> 8) % RT, chl = (e >> 8) / RT;
      d[e] = x(16 * chl + 4 * (lane >> 4) + el, 16 * ct + (lane & 15));
    }
  }
  if (NQ > 0) {  // rank quads of the last tile
    float* d = fb + fb_pq_off(rows, RP, NS) + (int64_t)ch16 * NQ * 64;
    for (int e = tid; e < (NR / 16) * NQ * 64; e += 256) {
      const int el = e & 3, jq = (e >> 2) & 3, g = (e >> 4) & 3, q = (e >> 6) % NQ,
                chl = (e >> 6) / NQ;
      d[e] = x(16 * chl + 4 * g + el, RP - 16 + 4 * q + jq);
    }
  }
  if (hb) {
    __bf16* h = reinterpret_cast<__bf16*>(hb);
    const int NK = p.NK;
    const int64_t lo_off = hb_elems(rows, p.RK, RP);
    auto put = [&](int64_t at, float v) {
      const __bf16 hi = (__bf16)v;
      h[at] = hi;
      h[lo_off + at] = (__bf16)(v - (float)hi);
    };
    auto xr = [&](int i, int c) { return c < RP ? x(i, c) : 0.f; };  // RK may exceed RP
    {  // hA: per 16-row chunk, NK blocks of 64 lanes x 8
      const int64_t base = (int64_t)ch16 * NK * 512;
      for (int e = tid; e < (NR / 16) * NK * 512; e += 256) {
        const int el = e & 7, lane = (e >> 3) & 63, kb = (e >> 9) % NK, chl = (e >> 9) / NK;
        put(base + e, xr(16 * chl + (lane & 15), 32 * kb + 8 * (lane >> 4) + el));
      }
    }
    {  // hP: per 32-row chunk, two halves of NK blocks, rows permuted
      const int64_t base = rows * p.RK + (int64_t)ch32 * 2 * NK * 512;
      for (int e = tid; e < (NR / 32) * 2 * NK * 512; e += 256) {
        const int el = e & 7, lane = (e >> 3) & 63, kb = (e >> 9) % NK, t = ((e >> 9) / NK) & 1,
                  chl = (e >> 9) / (2 * NK);
        const int il = lane & 15, w = 8 * (il >> 2) + 4 * t + (il & 3);
        put(base + e, xr(32 * chl + w, 32 * kb + 8 * (lane >> 4) + el));
      }
    }
    {  // hB: per 32-row chunk, RT tiles of 64 lanes x 8
      const int64_t base = 2 * rows * p.RK + (int64_t)ch32 * RT * 512;
      for (int e = tid; e < (NR / 32) * RT * 512; e += 256) {
        const int el = e & 7, lane = (e >> 3) & 63, ct = (e >> 9) % RT, chl = (e >> 9) / RT;
        put(base + e, x(32 * chl + 8 * (lane >> 4) + el, 16 * ct + (lane & 15)));
      }
    }
  }
}

// v_mfma_f32_4x4x1f32: 16 independent 4x4x1 products; block b = l/4 takes
// A_b[i] from lane 4b + i and B_b[j] from lane 4b + j, and D_b[i][j] lands in
// lane 4b + j, element i.
__device__ __forceinline__ f4 mfma4x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}


// S-pass statistics: the work-group's sums of Lambda^2, |S|, nnz(S) and (in
// rounds whose lambda is not the target) the Huber sum H_{lambda_target}(R)
// over its NW waves, added in wave order, into p.spart.
template <int NW>
__device__ __forceinline__ void spass_stats(const DevParams& p, int ci, int b, double sl2,
                                            double sl1, uint32_t nnz, double shb) {
  const int tid = threadIdx.x, lane = tid & 63;
  __shared__ double sred[NW][4];
  sl2 = wave_sum(sl2);
  sl1 = wave_sum(sl1);
  shb = wave_sum(shb);
  const int wv = tid >> 6;
  if (lane == 0) {
    sred[wv][0] = sl2;
    sred[wv][1] = sl1;
    sred[wv][2] = (double)nnz;
    sred[wv][3] = shb;
  }
  __syncthreads();
  if (tid == 0) {
    double* o = p.spart + ((int64_t)ci * p.nrb + b) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) t += sred[k][q];
      o[q] = t;
    }
  }
}

// H_lt(R) of one residual entry (Appendix A.2's Huber function): R^2 / 2
// within the threshold, lt |R| - lt^2 / 2 beyond it. By the Huber identity it
// is the least value over S of (R - S)^2 / 2 + lt |S|.
__device__ __forceinline__ float huber1(float R, float lt) {
  // With c = min(|R|, lt): c (|R| - c / 2) is R^2 / 2 for |R| <= lt and
  // lt |R| - lt^2 / 2 beyond (three instructions, no select).
  const float a = fabsf(R), c = fminf(a, lt);
  return c * fmaf(-0.5f, c, a);
}

// ---------------------------------------------------------------------------
// Finalize: G = U^T U + rho I from the Gram partials, G^{-1} by the FP64
// sweep, and (record = 1) the round statistics. It runs either as one
// standalone work-group (k_finalize) or folded into the next round's V-pass
// launch as two extra work-groups (Gram and inverse; statistics) whose record
// the V finish then assembles. Both forms run the same functions on
// kFinThreads threads, so they give bitwise the same results.
// ---------------------------------------------------------------------------

// Gram of the new U (slot gi) from its row-block partials into LDS A (r x r).
static __device__ void fin_gram(const DevParams& p, int gi, double* A) {
  const int r = p.r, RP = p.RP;
  const int64_t RR = (int64_t)RP * RP;
  const double* gp = p.gram_part + (int64_t)gi * p.nub * RR;
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    const int a = e / r, b = e - (e / r) * r;
    A[e] = sum_strided(gp + a * RP + b, p.nub, RR);
  }
}

// Round statistics from the partials of the round's kernels; result in
// out[0..6] of thread 0: ||Lambda||^2, ||S||_1, nnz(S), ||V||^2, ||dU||^2,
// the U penalty of the objective at the round's start, and the Huber sum at
// the target lambda (rounds at another lambda only).
static __device__ void fin_stats(const DevParams& p, double* out) {
  __shared__ double red[kFinThreads / 64][6];
  const int tid = threadIdx.x;
  if (tid < kFinThreads) {
    const int nsp = p.E * p.nrb;
    double l2 = block_strided_sum(nsp, [&](int k) { return p.spart[(int64_t)k * 4 + 0]; }, kFinThreads);
    double l1 = block_strided_sum(nsp, [&](int k) { return p.spart[(int64_t)k * 4 + 1]; }, kFinThreads);
    double nz = block_strided_sum(nsp, [&](int k) { return p.spart[(int64_t)k * 4 + 2]; }, kFinThreads);
    double hb = block_strided_sum(nsp, [&](int k) { return p.spart[(int64_t)k * 4 + 3]; }, kFinThreads);
    double vsq = block_strided_sum(p.ngroups, [&](int k) { return p.gv_tr[k]; }, kFinThreads);
    double du = block_strided_sum(p.nub, [&](int k) { return p.upart[k]; }, kFinThreads);
    l2 = wave_sum(l2);
    l1 = wave_sum(l1);
    nz = wave_sum(nz);
    vsq = wave_sum(vsq);
    du = wave_sum(du);
    hb = wave_sum(hb);
    if ((tid & 63) == 0) {
      red[tid >> 6][0] = l2;
      red[tid >> 6][1] = l1;
      red[tid >> 6][2] = nz;
      red[tid >> 6][3] = vsq;
      red[tid >> 6][4] = du;
      red[tid >> 6][5] = hb;
    }
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 0; q < 5; ++q) {
      double t = 0.0;
      for (int k = 0; k < kFinThreads / 64; ++k) t += red[k][q];
      out[q] = t;
    }
    double ureg;
    if (p.K == 1) {
      ureg = 0.5 * p.rho * p.dstate->u_sq;
    } else {
      ureg = 0.0;
      for (int i = 0; i < p.E; ++i) ureg += 0.5 * p.clients[i].c * p.ucl_sq[i];
    }
    out[5] = ureg;
    double t = 0.0;
    for (int k = 0; k < kFinThreads / 64; ++k) t += red[k][5];
    out[6] = t;
  }
}

// G^{-1} of the Gram in LDS A (adds rho I) into Ginv slot gi; returns
// tr(U^T U) (valid in every thread).
template <int EPT, bool BATCH = (EPT <= 4)>
static __device__ double fin_inverse(const DevParams& p, double* A, double* Ginv, int64_t g_stride, int gi) {
  __shared__ double tr_sh;
  const int tid = threadIdx.x, r = p.r, RP = p.RP;
  const int64_t RR = (int64_t)RP * RP;
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < r; ++k) t += A[k * r + k];
    tr_sh = t;
  }
  __syncthreads();
  for (int k = tid; k < r; k += blockDim.x) A[k * r + k] += p.rho;
  __syncthreads();
  spd_inverse<EPT, BATCH>(A, r, r);
  double* Gout = Ginv + (int64_t)gi * g_stride;
  for (int e = tid; e < RR; e += blockDim.x) {
    const int a = e / RP, b = e % RP;
    Gout[e] = (a < r && b < r) ? A[a * r + b] : 0.0;
  }
  return tr_sh;
}

// Round record from the statistics and tr(U^(t+1)T U^(t+1)) (one thread).
static __device__ void fin_record(const DevParams& p, const double* stats, double tr) {
  const int64_t t = p.dstate->t;
  StatsRec rec;
  rec.t = (double)t;
  rec.objective = 0.5 * stats[0] + 0.5 * p.rho * stats[3] + (double)p.lam_rec * stats[1] + stats[5];
  // At the target lambda the objective with S = soft(R) is the Huber form
  // itself (Huber identity); at another lambda the S-pass summed it.
  rec.objective_target = p.lam_rec == p.lam_target
                             ? rec.objective
                             : stats[6] + 0.5 * p.rho * stats[3] + stats[5];
  rec.lambda_fro_sq = stats[0];
  rec.nnz = stats[2];
  rec.du_sq = stats[4];
  rec.u_sq = tr;
  rec.v_sq = stats[3];
  rec.l1 = stats[1];
  p.hist[t % kHist] = rec;
  p.dstate->t = t + 1;
  p.dstate->u_sq = tr;
}


// The same work folded into a V-pass launch, by work-group role: role 0 forms
// the Gram and its inverse (into Ginv slot 0, trace into dstate->u_sq_next),
// role 1 the statistics (into p.stat_part). Neither reads what the other or
// the streaming work-groups write; the V finish records the round. A: LDS
// of at least r x r doubles, which the launch shares with the streaming
// work-groups' own LDS (a work-group takes one role at a time, and a
// persistent one passes a barrier before its first tile).
static __device__ void finalize_role(const DevParams& p, double* Ginv, int role, double* A) {
  if (role == 0) {
    fin_gram(p, 0, A);
    __syncthreads();
    const double tr = fin_inverse<kFinEPT>(p, A, Ginv, 0, 0);
    if (threadIdx.x == 0) p.dstate->u_sq_next = tr;
  } else {
    __shared__ double st[7];
    fin_stats(p, st);
    if (threadIdx.x == 0)
      for (int q = 0; q < 7; ++q) p.stat_part[q] = st[q];
  }
}

// LDS pool of a V-pass launch (doubles): the folded finalize's r x r Gram
// (r <= RP <= kFoldMaxRP) or a streaming work-group's 64 x RP FP32 partial
// of W (wider ranks fold no finalize).
constexpr int vpass_pool_doubles(int RP) {
  return RP <= kFoldMaxRP && RP * RP > kVStreamCols * RP / 2 ? RP * RP : kVStreamCols * RP / 2;
}

// ===========================================================================
// Mixed precision (RPCA_FLAG_BF16). M, U and V enter the rank-r contractions
// as BF16 on v_mfma_f32_16x16x32_bf16 with FP32 accumulation; the residual,
// the soft-threshold, Lambda, the U-step terms and every statistic stay
// FP32/FP64 as in the FP32 passes, and the factors themselves stay FP32 (the
// BF16 operands are rounded copies written by the kernels that produce the
// factors). Each pass streams its own BF16 copy of M, laid out so that one
// 16-byte load per lane is exactly its MFMA operand: 2 B per entry and pass.
// ===========================================================================
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// Eight BF16 values of one 16-byte load as FP32 (a BF16 is the upper half of
// the FP32 of the same value; element 2k is the low half of word k).
__device__ __forceinline__ void unpack8(u4 u, float* x) {
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[2 * k] = __uint_as_float(w[k] << 16);
    x[2 * k + 1] = __uint_as_float(w[k] & 0xFFFF0000u);
  }
}
// Eight FP32 values rounded to nearest even into one BF16 operand.
__device__ __forceinline__ bf8 pack8(const float* x) {
  const f8 v = {x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7]};
  return __builtin_convertvector(v, bf8);
}


// Hi/lo split of eight FP32 values: hi = bf16(x), lo = bf16(x - hi), each
// rounded to nearest even, so that hi + lo carries 16 significand bits.
__device__ __forceinline__ void split8(const float* x, bf8& hi, bf8& lo) {
  hi = pack8(x);
  float r[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = x[e] - (float)hi[e];
  lo = pack8(r);
}
// (ah + al)(bh + bl) without the al bl term: three BF16 products, small ones
// first, with FP32 accumulation.
__device__ __forceinline__ f4 mfma3(bf8 ah, bf8 al, bf8 bh, bf8 bl, f4 c) {
  c = mfma_bf16(al, bh, c);
  c = mfma_bf16(ah, bl, c);
  return mfma_bf16(ah, bh, c);
}

// Work-groups of `kernel` (block threads, no dynamic LDS) that are resident
// on the current device at once, for the grid of a persistent launch; kept
// per kernel and device after the first query (0 if the runtime cannot
// tell). Kernels of one signature differ in their register and LDS use, so
// the cache is keyed by the kernel's address, not its type.
template <class K>
static int resident_groups(K kernel, int block) {
  struct Entry {
    const void* k;
    int dev, block, groups;
  };
  constexpr int kSlots = 256;
  static Entry cache[kSlots];
  static int used = 0;
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  const void* kp = reinterpret_cast<const void*>(kernel);
  {
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < used; ++i)
      if (cache[i].k == kp && cache[i].dev == dev && cache[i].block == block) return cache[i].groups;
  }
  int cus = 0, nb = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kp, block, 0) != hipSuccess)
    return 0;
  std::lock_guard<std::mutex> lock(mu);
  if (used < kSlots) cache[used++] = Entry{kp, dev, block, nb * cus};
  return nb * cus;
}

// Grid of a streaming pass over ntiles tiles: one work-group per tile, or
// (persistent) the resident work-groups, at most one per tile.
template <class K>
static int pass_groups(K kernel, int block, int ntiles, int persistent) {
  if (!persistent) return ntiles;
  const int res = resident_groups(kernel, block);
  return res > 0 && res < ntiles ? res : ntiles;
}

// Compile-time (RT, NS) dispatch for ranks up to kFoldMaxRP: NS = ceil(r/4)
// lies in [4 RT - 3, 4 RT]. (Wider ranks have launchers of their own, with
// NS = 4 RT.)
template <int RT, int NS, class F>
static hipError_t with_ns(int ns, F&& f) {
  if (ns == NS) return f(std::integral_constant<int, RT>{}, std::integral_constant<int, NS>{});
  if constexpr (NS < 4 * RT) return with_ns<RT, NS + 1>(ns, f);
  return hipErrorInvalidValue;
}
// Rank-tile dispatch (one to eight 16-rank tiles) for kernels whose code does
// not depend on NS.
template <class F>
static hipError_t with_rt(int RP, F&& f) {
  switch (RP / 16) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
  }
}
template <class F>
static hipError_t with_rank(const DevParams& p, F&& f) {
  switch (p.RP / 16) {
    case 1: return with_ns<1, 1>(p.NS, f);
    case 2: return with_ns<2, 5>(p.NS, f);
    case 3: return with_ns<3, 9>(p.NS, f);
    case 4: return with_ns<4, 13>(p.NS, f);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rpca
