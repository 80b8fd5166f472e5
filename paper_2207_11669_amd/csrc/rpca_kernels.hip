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
constexpr int kFinEPT = (kMaxRank * (kMaxRank + 1) / 2 + kFinThreads - 1) / kFinThreads;  // sweep entries per thread

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
// entries, indexed once. A pivot that is not positive (non-SPD or NaN input)
// turns the result into NaN, which the round statistics then expose.
template <int EPT>
__device__ void spd_inverse(double* A, int r, int ld) {
  __shared__ double xb[2][kMaxRank];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nl = r * (r + 1) / 2;
  int ei[EPT], ej[EPT];
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
  }
  if (tid < r) xb[0][tid] = A[tid * ld];
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    const int cur = k & 1, nxt = cur ^ 1;
    const double pv = xb[cur][k];
    if constexpr (EPT <= 4) {
      // The step's LDS reads go out together, before the pivot's reciprocal;
      // the three cases are then selects. (With many entries per thread the
      // held reads would cost more registers than the latency they save.)
      double xi[EPT], xj[EPT], aa[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        if (ei[q] >= 0) {
          xi[q] = xb[cur][ei[q]];
          xj[q] = xb[cur][ej[q]];
          aa[q] = A[ei[q] * ld + ej[q]];
        }
      const double pinv = pv > 0.0 ? recip_pos(pv) : NAN;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int i = ei[q], j = ej[q];
        if (i >= 0) {
          const double ci = i < k ? -xi[q] : xi[q];
          double v = aa[q] - ci * xj[q] * pinv;
          v = j == k ? -xi[q] * pinv : v;
          v = i == k ? (j == k ? pinv : xj[q] * pinv) : v;
          A[i * ld + j] = v;
          if (i == k + 1) xb[nxt][j] = v;
          if (j == k + 1) xb[nxt][i] = v;
        }
      }
    } else {
      const double pinv = pv > 0.0 ? recip_pos(pv) : NAN;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int i = ei[q], j = ej[q];
        if (i >= 0) {
          double v;
          if (i == k)
            v = (j == k) ? pinv : xb[cur][j] * pinv;
          else if (j == k)
            v = -xb[cur][i] * pinv;
          else {
            const double ci = i < k ? -xb[cur][i] : xb[cur][i];
            v = A[i * ld + j] - ci * xb[cur][j] * pinv;
          }
          A[i * ld + j] = v;
          if (i == k + 1) xb[nxt][j] = v;
          if (j == k + 1) xb[nxt][i] = v;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q)
    if (ei[q] > ej[q]) A[ej[q] * ld + ei[q]] = A[ei[q] * ld + ej[q]];
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

// ---------------------------------------------------------------------------
// V-pass, streaming part: W = (M_i - S_i)^T U_i partial sums over row splits.
// grid = (64-column groups x row splits, plus two finalize work-groups); 4
// waves. The U operands of a 16-row chunk (B packing, quads, and the previous
// U for the S rebuild) cost about as many loads as the chunk's M. With KG
// column groups per wave, a wave takes KG 16-column groups of the tile,
// which share the chunk's U operands in registers, and the KG waves on the
// same columns split the rows (wave phase q takes chunks q, q + KG, ...);
// their partial W are added in LDS in phase order at the end. KG = 1 keeps
// the four waves on distinct columns over the same rows, sharing U through
// L1 instead (fewer registers, more waves; better where the MFMA chains of
// a chunk, not its loads, set the pace). The autotuner picks KG.
// Lane l holds rows 4*(l/16)..+3 of column 16 g + l%16 (one float4 along the
// contiguous rows of the column-major block): element s of that float4 is the
// A operand of MFMA step s, and U supplies the B operand as one float4 of its
// B-operand packing. Accumulator: W[col 16 g + 4*(l/16)+v][rank 16*ct + l%16].
// MODE kSRecompute rebuilds S = soft(M - Uo Vo^T) of the previous round on the
// fly: its MFMA puts Uo rows on the A side and Vo^T on the B side, so the
// 16x16 residual tile comes out in exactly the float4 layout of M.
// ---------------------------------------------------------------------------
__device__ void finalize_role(const DevParams& p, double* Ginv, int role);
__device__ void fin_record(const DevParams& p, const double* stats, double tr);

template <int RT, int NS, int MODE, int KG>
__global__ __launch_bounds__(256) void k_vpass(DevParams p, const float* __restrict__ Ubase,
                                               int64_t u_stride, const float* __restrict__ Uold,
                                               const float* __restrict__ Vold,
                                               double* __restrict__ fin_Ginv, int fin) {
  constexpr int RP = 16 * RT;
  static_assert(NS >= 1 && NS <= 4 * RT, "NS = ceil(r / 4) must fit the rank tiles");
  // W's last rank tile in 4x4 blocks when it holds at most 12 ranks.
  constexpr int NQ = nquads(RP, NS), RTF = NQ ? RT - 1 : RT;
  constexpr int kG = KG;                 // column groups per wave
  constexpr int kPh = KG;                // row phases (waves per column set)
  static_assert(KG == 1 || KG == 2 || KG == 4, "column groups per wave");
  // fin = 1: the first two work-groups run the previous round's finalize
  // (Gram inverse into fin_Ginv slot 0; round statistics) while the others
  // stream; nothing in this kernel reads what they write.
  int bid = (int)blockIdx.x;
  if (fin) {
    if (bid < 2) {
      finalize_role(p, fin_Ginv, bid);
      return;
    }
    bid -= 2;
  }
  const int gx = bid % p.ng64, gy = bid / p.ng64;
  const VTile vt = p.vg64[gx];
  const ClientDev& cl = vt.cl;
  const float* __restrict__ U = Ubase + (int64_t)vt.client * u_stride;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  // Wave-uniform; readfirstlane lets the compiler keep the buffer resources
  // built from it in scalar registers (no per-load uniformity loops).
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cset = w % (4 / kPh), ph = w / (4 / kPh);  // column set, row phase
  const int jw = vt.j0 + 16 * kG * cset;               // first column of this wave
  const float lam = p.lam;

  const float* gUpb_raw = U + fb_pb_off(p.MP, RP, NS);
  const float* gUopa_raw = (MODE == kSRecompute) ? Uold + fb_pa_off(p.MP, RP) : gUpb_raw;
  float vb[kG][NS];  // B operand of the S rebuild: Vo[col jw + 16 g + l%16][rank (l/16)*NS + s]
  if (MODE == kSRecompute) {
    const GLOBAL float* Vopa = gptr(v_fb(Vold, p.NVP, RP)) + fb_pa_off(p.NVP, RP);
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int vch = (cl.vrow0 + jw + 16 * g) >> 4;
#pragma unroll
      for (int s = 0; s < NS; ++s) vb[g][s] = Vopa[((int64_t)vch * NS + s) * 64 + lane];
    }
  }

  const int rbeg = gy * p.vsplit_rows;
  const int rend = min(p.m, rbeg + p.vsplit_rows);
  const int nch = (rend - rbeg + 15) >> 4;
  const int nk = (nch - ph + kPh - 1) / kPh;  // this wave's chunks ph, ph + kPh, ...
  f4 acc[kG][RTF > 0 ? RTF : 1], accq[kG][NQ > 0 ? NQ : 1];
#pragma unroll
  for (int g = 0; g < kG; ++g) {
#pragma unroll
    for (int ct = 0; ct < RTF; ++ct) acc[g][ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NQ; ++q) accq[g][q] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // M (and stored S) through one buffer resource per 16-column group: columns
  // past n_i lie beyond its range and read 0; rows are clamped to the last
  // float4 of the column and masked when used. U operands are packed and
  // always in range: lane offset plus a scalar chunk offset.
  const int mlast4 = (p.m - 1) & ~3;
  rsrc_t rM[kG], rS[kG];
#pragma unroll
  for (int g = 0; g < kG; ++g) {
    const int j0 = jw + 16 * g;
    rM[g] = make_rsrc(cl.M + (int64_t)min(j0, cl.n) * cl.ldm, block_bytes_from(cl.n, j0, cl.ldm));
    rS[g] = rM[g];
    if (MODE == kSStored)
      rS[g] = make_rsrc(p.S + cl.s_off + (int64_t)min(j0, cl.n) * p.lds, block_bytes_from(cl.n, j0, p.lds));
  }
  const uint32_t vM = (uint32_t)(li * cl.ldm) * 4u, vS = (uint32_t)(li * p.lds) * 4u;
  const rsrc_t rUb = make_rsrc(gUpb_raw, (uint32_t)(p.MP * RP * 4));
  const rsrc_t rUq = make_rsrc(U + fb_pq_off(p.MP, RP, NS), (uint32_t)(p.MP * 4 * NQ * 4));
  const uint32_t vq_off = (uint32_t)(((lane >> 4) * 4 + (lane & 3)) * 16);
  const rsrc_t rUa = make_rsrc(gUopa_raw, (uint32_t)(p.MP * 4 * NS * 4));

  // Operands of one 16-row chunk; kVDepth chunks are kept in flight (vector
  // loads complete in order, so everything a chunk needs is issued together).
  struct Chunk {
    f4 m[kG], s[kG];          // M (and stored S) rows 4*(l/16)..+3 of column 16 g + l%16
    f4 u[RTF > 0 ? RTF : 1];  // U^T operand: U[row][rank 16*ct + l%16] for the 4 rows
    f4 uq[NQ > 0 ? NQ : 1];   // quads: U[row][rank RP - 16 + 4 q + l%4] for the 4 rows
    float uo[NS];             // previous U, A operand of the S rebuild: Uo[row l%16][rank g*NS + s]
  };
  // Two chunks in flight per wave: deeper rings measured slower at r = 20
  // (more outstanding loads per compute unit, no better latency cover).
  constexpr int kVDepth = 2;
  Chunk ring[kVDepth];
  auto load_chunk = [&](Chunk& c, int k) {
    const int row0 = rbeg + ((ph + kPh * k) << 4);
    const uint32_t rowb = (uint32_t)min(row0 + 4 * lg, mlast4) * 4u;
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      c.m[g] = bload4(rM[g], vM + rowb, 0);
      if (MODE == kSStored) c.s[g] = bload4(rS[g], vS + rowb, 0);
    }
    const uint32_t chg = (uint32_t)(row0 >> 4);
#pragma unroll
    for (int ct = 0; ct < RTF; ++ct)
      c.u[ct] = bload4(rUb, (uint32_t)lane * 16u, ((chg * RT + ct) * 64u) * 16u);
#pragma unroll
    for (int q = 0; q < NQ; ++q) c.uq[q] = bload4(rUq, vq_off, (chg * NQ + q) * 256u);
    if (MODE == kSRecompute) {
#pragma unroll
      for (int s = 0; s < NS; ++s) c.uo[s] = bload(rUa, (uint32_t)lane * 4u, ((chg * NS + s) * 64u) * 4u);
    }
  };
  auto compute_chunk = [&](const Chunk& c, int k) {
    // Columns past n_i read 0 from M (and S) and have zero rows in the old V,
    // so they give d = 0 without a mask; only the chunk that crosses row m
    // (whose last float4 may hold the caller's padding rows) is masked.
    const int row0 = rbeg + ((ph + kPh * k) << 4);
    const int row = row0 + 4 * lg;
    const bool tail = row0 + 16 > p.m;  // wave-uniform
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      f4 d;
      if (MODE == kSRecompute) {
        f4 a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NS; ++s) a1 = mfma4(c.uo[s], vb[g][s], a1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float R = c.m[g][e] - a1[e];
          const float Sv = R - __builtin_amdgcn_fmed3f(R, -lam, lam);
          d[e] = c.m[g][e] - Sv;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) d[e] = c.m[g][e] - (MODE == kSStored ? c.s[g][e] : 0.f);
      }
      if (tail) {
#pragma unroll
        for (int e = 0; e < 4; ++e) d[e] = row + e < p.m ? d[e] : 0.f;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int ct = 0; ct < RTF; ++ct) acc[g][ct] = mfma4(d[s], c.u[ct][s], acc[g][ct]);
#pragma unroll
        for (int q = 0; q < NQ; ++q) accq[g][q] = mfma4x4(d[s], c.uq[q][s], accq[g][q]);
      }
    }
  };
  if (nk > 0) {
    // Uniform loop: every iteration loads (the chunk index is clamped to the
    // wave's last chunk, whose addresses are then cache hits), so the wait
    // counts stay exact and kVDepth - 1 chunks remain in flight at every wait.
    const int nkp = (nk + kVDepth - 1) / kVDepth * kVDepth;
    // The prologue issues the ring in slot order (fenced like the loop body),
    // so that at the loop head slot 0 holds the oldest loads on every path.
#pragma unroll
    for (int d = 0; d < kVDepth; ++d) {
      load_chunk(ring[d], min(d, nk - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int k0 = 0; k0 < nkp; k0 += kVDepth) {
#pragma unroll
      for (int d = 0; d < kVDepth; ++d) {
        const int k = k0 + d;
        if (k < nk) compute_chunk(ring[d], k);  // wave-uniform
        // Keep the refill at this point of the program: left alone, the
        // scheduler sinks loads towards their first use and the ring
        // collapses to a single chunk in flight.
        __builtin_amdgcn_sched_barrier(0);
        load_chunk(ring[d], min(k + kVDepth, nk - 1));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // Quads: block b = l/4 summed rows 4 (b/4) + s of columns 4 (b%4) + i; the
  // four row groups (lanes l, l ^ 16, l ^ 32, l ^ 48) are added first.
#pragma unroll
  for (int g = 0; g < kG; ++g)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float x = accq[g][q][i];
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        accq[g][q][i] = x;
      }
  // Partial W of the waves, added in LDS in row-phase order; the
  // work-group then writes its partial of the 64 columns.
  __shared__ float red[kVStreamCols][RP];
  const int c0 = 16 * kG * cset;
  for (int q0 = 0; q0 < kPh; ++q0) {
    if (ph == q0) {
#pragma unroll
      for (int g = 0; g < kG; ++g) {
#pragma unroll
        for (int ct = 0; ct < RTF; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float& x = red[c0 + 16 * g + 4 * lg + v][16 * ct + li];
            x = q0 == 0 ? acc[g][ct][v] : x + acc[g][ct][v];
          }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (lane < 16) {
              float& x = red[c0 + 16 * g + 4 * (lane >> 2) + i][16 * RTF + 4 * q + (lane & 3)];
              x = q0 == 0 ? accq[g][q][i] : x + accq[g][q][i];
            }
      }
    }
    __syncthreads();
  }
  GLOBAL float* wp = gptr_w(p.Wpart) + ((int64_t)gy * p.NVP + cl.vrow0 + vt.j0) * RP;
  for (int e = tid; e < kVStreamCols * RP; e += blockDim.x) {
    const int c = e % RP;
    // Ranks past the quads are never accumulated: zero (the padding ranks of
    // W are read by the V finish only through zero rows of G^{-1}).
    wp[e] = (NQ && c >= 16 * RTF + 4 * NQ) ? 0.f : red[e / RP][c];
  }
}

// ---------------------------------------------------------------------------
// V-pass, finalize: one work-group per 32 columns. W = sum of the row-split
// partials (fixed order, FP64), V = W (U^T U + rho I)^{-1} (eq. "condition1"),
// rounded to FP32 once and written in both layouts, plus the partial V^T V of
// these columns.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_vfinal(DevParams p, const double* __restrict__ Gbase,
                                                int64_t g_stride, int rec) {
  constexpr int RP = 16 * RT;
  // rec = 1: record the previous round, whose finalize ran in the V-pass.
  if (rec && blockIdx.x == 0 && threadIdx.x == 0) {
    double st[6];
    for (int q = 0; q < 6; ++q) st[q] = p.stat_part[q];
    fin_record(p, st, p.dstate->u_sq_next);
  }
  __shared__ double wd[kVCols][RP + 1];
  __shared__ double gl[RP * RP];
  const VGroup vg = p.vgroups[blockIdx.x];
  const double* __restrict__ Gi = Gbase + (int64_t)vg.client * g_stride;
  const int tid = threadIdx.x;
  const int vrow = vg.vrow;
  const int64_t split_stride = (int64_t)p.NVP * RP;
  constexpr int kPer = (kVCols * RP + 255) / 256;
  constexpr int kGPer = (RP * RP + 255) / 256;
  {
    // All of a thread's loads (kWB row splits of each of its W entries, and
    // its share of G^{-1}) are issued before any is used; splits are summed
    // in increasing order. Wider ranks batch fewer splits, which keeps the
    // batch's addresses within the register file.
    double gv_[kGPer];
#pragma unroll
    for (int q = 0; q < kGPer; ++q) {
      const int e = tid + q * 256;
      gv_[q] = Gi[e];  // RP^2 is a multiple of 256
    }
    double acc[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
    constexpr int kWB = RT <= 2 ? 8 : 4;
    for (int s0 = 0; s0 < p.vsplit; s0 += kWB) {
      float wv[kPer][kWB];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int e = tid + q * 256;
        const int j = e / RP, c = e % RP;
        const float* src = p.Wpart + (int64_t)(vrow + j) * RP + c;
        // Every load is unconditional (splits past the last re-read it and
        // are masked afterwards): a load under a branch gets its own wait,
        // which serialised the batch.
#pragma unroll
        for (int u = 0; u < kWB; ++u) {
          const float x = src[(int64_t)min(s0 + u, p.vsplit - 1) * split_stride];
          wv[q][u] = s0 + u < p.vsplit ? x : 0.f;
        }
      }
#pragma unroll
      for (int q = 0; q < kPer; ++q)
#pragma unroll
        for (int u = 0; u < kWB; ++u) acc[q] += (double)wv[q][u];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * 256;
      if (e < kVCols * RP) wd[e / RP][e % RP] = acc[q];
    }
#pragma unroll
    for (int q = 0; q < kGPer; ++q) {
      const int e = tid + q * 256;
      if (e < RP * RP) gl[e] = gv_[q];
    }
  }
  __syncthreads();
  // V = W G^{-1}: thread tid holds entries e = tid + 256 q, (j, c) =
  // (e / RP, e % RP), as kPer sums in registers over k in increasing order.
  // When RP divides 256 all of a thread's entries share c, so each G^{-1}
  // entry it reads feeds kPer FMAs.
  static_assert(kPer * 256 == kVCols * RP, "V finish thread mapping");
  float vres[kPer];
  {
    double sv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) sv[q] = 0.0;
#pragma unroll 2
    for (int k = 0; k < p.r; ++k) {
      if constexpr (256 % RP == 0) {
        const double g = gl[k * RP + tid % RP];
#pragma unroll
        for (int q = 0; q < kPer; ++q) sv[q] += wd[(tid + 256 * q) / RP][k] * g;
      } else {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
          const int e = tid + 256 * q;
          sv[q] += wd[e / RP][k] * gl[k * RP + e % RP];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + 256 * q, j = e / RP, c = e % RP;
      vres[q] = (j < vg.ncols && c < p.r) ? (float)sv[q] : 0.f;
    }
  }
  __syncthreads();
  // V to LDS and its row-major copy (consecutive threads, consecutive ranks),
  // then the packed layouts from LDS, each walked in its own order.
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * 256, j = e / RP, c = e % RP;
    wd[j][c] = (double)vres[q];
    p.V[(int64_t)(vrow + j) * RP + c] = vres[q];
  }
  __syncthreads();
  factor_store_rows<RT, kVCols>(v_fb(p.V, p.NVP, RP), p.bf16 ? v_hb(p.V, p) : nullptr, p.NVP, p,
                                vrow, [&](int i, int c) { return (float)wd[i][c]; });
  // Partial V^T V of these columns: thread (ta, tb) = (tid / 16, tid % 16)
  // forms the RT x RT block of entries (RT ta + x, RT tb + y), each a sum over
  // the 32 columns in order (each LDS read feeds RT FMAs).
  double* gv = p.gv_part + (int64_t)blockIdx.x * RP * RP;
  {
    const int a0 = RT * (tid >> 4), b0 = RT * (tid & 15);
    double sg[RT][RT];
#pragma unroll
    for (int x = 0; x < RT; ++x)
#pragma unroll
      for (int y = 0; y < RT; ++y) sg[x][y] = 0.0;
#pragma unroll 2
    for (int j = 0; j < kVCols; ++j) {
      double va[RT], vb[RT];
#pragma unroll
      for (int x = 0; x < RT; ++x) {
        va[x] = wd[j][a0 + x];
        vb[x] = wd[j][b0 + x];
      }
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < RT; ++y) sg[x][y] += va[x] * vb[y];
    }
#pragma unroll
    for (int x = 0; x < RT; ++x)
#pragma unroll
      for (int y = 0; y < RT; ++y) gv[(a0 + x) * RP + b0 + y] = sg[x][y];
  }
}

// ---------------------------------------------------------------------------
// Per-client r x r factors for the closed-form U step:
//   A_i = (V_i^T V_i + c_i I)^{-1},  B_i = V_i^T V_i A_i,  c_i = rho n_i / n.
// One work-group per client; FP64 throughout.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_client_factor(DevParams p) {
  __shared__ double A[kMaxRank * kMaxRank], G[kMaxRank * kMaxRank];
  const int r = p.r, RP = p.RP;
  const int64_t RR = (int64_t)RP * RP;
  const ClientDev cl = p.clients[blockIdx.x];
  const int tid = threadIdx.x;
  if (cl.g1 - cl.g0 <= 16) {
    // One block of groups: one batch of loads per entry.
    for (int e = tid; e < r * r; e += blockDim.x) {
      const int a = e / r, b = e % r;
      const double s = sum_strided(p.gv_part + (int64_t)cl.g0 * RR + a * RP + b, cl.g1 - cl.g0, RR);
      G[e] = s;
      A[e] = s + (a == b ? cl.c : 0.0);
    }
  } else {
    // G = V_i^T V_i from the V finish's per-group partials, which are
    // symmetric bit for bit (each partial multiplies the same two factors
    // both ways round): the lower triangle is summed and mirrored. Sums run
    // in blocks of 16 groups as in sum_strided, same bits, but all of a
    // thread's entries load together, 8 groups at a time, with no load
    // under a branch: out-of-range groups and entries re-read a valid,
    // finite partial and are multiplied by 0 (a select would let the
    // compiler move the load into a branch of its own, with its own wait).
    constexpr int kCE = 3;  // 1024 threads x 3 >= 64 x 65 / 2
    const int nl = r * (r + 1) / 2, ng = cl.g1 - cl.g0;
    const double* __restrict__ gp = p.gv_part + (int64_t)cl.g0 * RR;
    int ia[kCE], ib[kCE];
    double s[kCE];
#pragma unroll
    for (int q = 0; q < kCE; ++q) {
      const int e = tid + q * 1024;
      int a = -1, b = 0;
      if (e < nl) {
        a = (int)((sqrtf(8.f * (float)e + 1.f) - 1.f) * 0.5f);
        while (a * (a + 1) / 2 > e) --a;
        while ((a + 1) * (a + 2) / 2 <= e) ++a;
        b = e - a * (a + 1) / 2;
      }
      ia[q] = a;
      ib[q] = b;
      s[q] = 0.0;
    }
    for (int g0 = 0; g0 < ng; g0 += 16) {
      double t[kCE];
#pragma unroll
      for (int q = 0; q < kCE; ++q) t[q] = 0.0;
#pragma unroll
      for (int h = 0; h < 16; h += 8) {
        double v[kCE][8];
#pragma unroll
        for (int q = 0; q < kCE; ++q)
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int g = g0 + h + u;
            const double x = gp[(int64_t)min(g, ng - 1) * RR + max(ia[q], 0) * RP + ib[q]];
            v[q][u] = x * (double)(ia[q] >= 0 && g < ng);
          }
#pragma unroll
        for (int q = 0; q < kCE; ++q)
#pragma unroll
          for (int u = 0; u < 8; ++u) t[q] += v[q][u];
      }
#pragma unroll
      for (int q = 0; q < kCE; ++q) s[q] += t[q];
    }
#pragma unroll
    for (int q = 0; q < kCE; ++q)
      if (ia[q] >= 0) {
        const int a = ia[q], b = ib[q];
        G[a * r + b] = s[q];
        G[b * r + a] = s[q];
        A[a * r + b] = s[q] + (a == b ? cl.c : 0.0);
        A[b * r + a] = s[q] + (a == b ? cl.c : 0.0);
      }
  }
  __syncthreads();
  spd_inverse<3>(A, r, r);  // 1024 threads x 3 >= 64 x 65 / 2
  double* Af = p.Afac + (int64_t)blockIdx.x * RR;
  double* Bf = p.Bfac + (int64_t)blockIdx.x * RR;
  for (int e = tid; e < RR; e += blockDim.x) {
    const int a = e / RP, b = e % RP;
    double av = 0.0, bv = 0.0;
    if (a < r && b < r) {
      av = A[a * r + b];
      for (int k = 0; k < r; ++k) bv += G[a * r + k] * A[k * r + b];
    }
    Af[e] = av;
    Bf[e] = bv;
  }
}

// S-pass statistics: the work-group's sums of Lambda^2, |S| and nnz(S) over
// its NW waves, added in wave order, into p.spart.
template <int NW>
__device__ __forceinline__ void spass_stats(const DevParams& p, int ci, int b, double sl2,
                                            double sl1, uint32_t nnz) {
  const int tid = threadIdx.x, lane = tid & 63;
  __shared__ double sred[NW][3];
  sl2 = wave_sum(sl2);
  sl1 = wave_sum(sl1);
  const int wv = tid >> 6;
  if (lane == 0) {
    sred[wv][0] = sl2;
    sred[wv][1] = sl1;
    sred[wv][2] = (double)nnz;
  }
  __syncthreads();
  if (tid == 0) {
    double* o = p.spart + ((int64_t)ci * p.nrb + b) * 4;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) t += sred[k][q];
      o[q] = t;
    }
    o[3] = 0.0;
  }
}

// S-pass epilogue of the FP32 form (NW waves): the client's U-step term for the work-group's 128 rows from P = Lambda V_i and
// U_i staged in LDS (Lemma 2 proof for the gradient, argmin_U L_i for the
// closed form):
//   GRAD   T = U_i - eta (c_i U_i - P)
//   CLOSED T = P A_i + U_i B_i,  A_i = (V_i^T V_i + c_i I)^{-1}, B_i = V_i^T V_i A_i
// in FP64, stored FP32 into the client's slot of p.P; then the statistics.
template <int RP, int NW>
__device__ __forceinline__ void spass_terms_and_stats(const DevParams& p, const ClientDev& cl, int b,
                                                      const float (*ptile)[RP + 1],
                                                      const float (*utile)[RP + 1],
                                                      const double (*fab)[RP * RP], bool closed,
                                                      double sl2, double sl1, uint32_t nnz) {
  const int tid = threadIdx.x;
  const int ci = cl.idx;
  const int row0 = b * kSRows;
  float* Ti = p.P + (int64_t)ci * RP * p.MP;
  const double eta = eta_of_round(p, p.dstate->t);
  const double cc = cl.c;
  // Thread: one row, eight rank columns (register blocking: each LDS read of
  // P or U feeds eight FMAs).
  for (int e = tid; e < kSRows * (RP / 8); e += blockDim.x) {
    const int rl = e % kSRows, c0 = (e / kSRows) * 8;
    double t[8];
    if (closed) {
#pragma unroll
      for (int j = 0; j < 8; ++j) t[j] = 0.0;
      for (int k = 0; k < p.r; ++k) {
        const double pk = (double)ptile[rl][k], uk = (double)utile[rl][k];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          t[j] = fma(pk, fab[0][k * RP + c0 + j], fma(uk, fab[1][k * RP + c0 + j], t[j]));
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double u = utile[rl][c0 + j];
        t[j] = u - eta * (cc * u - (double)ptile[rl][c0 + j]);
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      Ti[(int64_t)(c0 + j) * p.MP + row0 + rl] = c0 + j < p.r ? (float)t[j] : 0.f;
  }

  spass_stats<NW>(p, ci, b, sl2, sl1, nnz);
}

// ---------------------------------------------------------------------------
// S-pass: one work-group per (128-row block, client); each of its 4 row waves
// owns 32 rows (two 16-row tiles) and sweeps the client's columns 16 at a time,
// alone (NPH = 1, 256 threads) or with a partner wave taking alternate column
// chunks (NPH = 2, 512 threads).
// MFMA 1 forms (U V^T)^T for a 16x16 tile with V as the A operand and U^T as
// the B operand, so lane l ends up with row l%16 and columns 4*(l/16)+v.
// That is exactly the A-operand layout of MFMA 2 (P += Lambda V, contraction
// over columns), so Lambda goes from the accumulator to the next MFMA without
// any data movement. M is read and S written one dword per lane per column
// (16 consecutive rows per column per instruction).
// The contraction index of MFMA 1 is split as k-group g = l/16 taking rank
// indices g*NS + s, s < NS = ceil(r/4), so no padding steps run for r % 16.
// ---------------------------------------------------------------------------
template <int RT, int NS, bool STORE, int NPH>
__global__ __launch_bounds__(256 * NPH) void k_spass(DevParams p, const float* __restrict__ Ubase,
                                               int64_t u_stride, float* __restrict__ Sout,
                                               int64_t lds_out, int emit_only, int client_base) {
  constexpr int RP = 16 * RT;
  static_assert(NS >= 1 && NS <= 4 * RT, "NS = ceil(r / 4) must fit the rank tiles");
  // P's last rank tile in 4x4 blocks when it holds at most 12 ranks.
  constexpr int NQ = nquads(RP, NS), RTF = NQ ? RT - 1 : RT;
  // Clients run widest first (longest work-groups dispatched earliest), except
  // for the S emission of a client range.
  const int b = blockIdx.x;
  const ClientDev cl = emit_only ? p.clients[client_base + (int)blockIdx.y]
                                 : p.clients_lpt[blockIdx.y];
  const int ci = cl.idx;
  const float* __restrict__ U = Ubase + (int64_t)ci * u_stride;
  const int tid = threadIdx.x, lane = tid & 63, w = (tid >> 6) & 3;
  // NPH column phases of four waves each, phase q taking chunks q, q + NPH, ...
  // Wave-uniform (waves 0-3: phase 0, waves 4-7: phase 1); readfirstlane tells
  // the compiler so, which keeps the chunk addressing in scalar registers.
  const int phase = NPH == 2 ? __builtin_amdgcn_readfirstlane(tid >> 8) : 0;
  const int li = lane & 15, lg = lane >> 4;
  const int arow0 = b * kSRows + w * 32;

  float ub[2][NS];  // MFMA 1 B operand: U[row arow0 + 16 rt + l%16][rank (l/16)*NS + s]
  {
    const GLOBAL float* Upa = gptr(U) + fb_pa_off(p.MP, RP);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t ch = (arow0 + 16 * rt) >> 4;
#pragma unroll
      for (int s = 0; s < NS; ++s) ub[rt][s] = Upa[(ch * NS + s) * 64 + lane];
    }
  }
  f4 accp[2][RTF > 0 ? RTF : 1], accq[2][NQ > 0 ? NQ : 1];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
#pragma unroll
    for (int ct = 0; ct < RTF; ++ct) accp[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NQ; ++q) accq[rt][q] = f4{0.f, 0.f, 0.f, 0.f};
  }

  // Epilogue operands that do not depend on the sweep: the closed-form
  // factors A_i and B_i are fetched now (into registers, stored to LDS once
  // the ring's first loads are in flight), so the epilogue waits on no memory.
  __shared__ float ptile[kSRows][RP + 1];
  __shared__ float utile[kSRows][RP + 1];
  __shared__ double fab[2][RP * RP];
  const bool closed = p.u_mode != 0;
  constexpr int kFabPer = (RP * RP + 256 * NPH - 1) / (256 * NPH);
  double fa[kFabPer], fbv[kFabPer];
  if (!emit_only && closed) {
    const double* __restrict__ Af = p.Afac + (int64_t)ci * RP * RP;
    const double* __restrict__ Bf = p.Bfac + (int64_t)ci * RP * RP;
#pragma unroll
    for (int q = 0; q < kFabPer; ++q) {
      const int e = tid + q * 256 * NPH;
      fa[q] = e < RP * RP ? Af[e] : 0.0;
      fbv[q] = e < RP * RP ? Bf[e] : 0.0;
    }
  }

  double sl2 = 0.0, sl1 = 0.0;
  uint32_t nnz = 0;  // wave-uniform count of nonzero S entries
  const float lam = p.lam;
  GLOBAL float* Sblk = STORE ? gptr_w(Sout) + cl.col0 * lds_out : nullptr;
  // V operands: packed, always in range (lane offset + scalar chunk offset).
  const rsrc_t rVa = make_rsrc(v_fb(p.V, p.NVP, RP) + fb_pa_off(p.NVP, RP), (uint32_t)(p.NVP * 4 * NS * 4));
  const rsrc_t rVb = make_rsrc(v_fb(p.V, p.NVP, RP) + fb_pb_off(p.NVP, RP, NS), (uint32_t)(p.NVP * RP * 4));
  const rsrc_t rVq = make_rsrc(v_fb(p.V, p.NVP, RP) + fb_pq_off(p.NVP, RP, NS), (uint32_t)(p.NVP * 4 * NQ * 4));
  const uint32_t vq_off = (uint32_t)(((lane >> 4) * 4 + (lane & 3)) * 16);
  // M: one buffer resource per 16-column chunk (base at the chunk's first
  // column, range = the rest of the block, at most kChunkRange), fixed per-lane
  // offsets. Columns past n_i fall outside the range and rows past m get an
  // offset beyond any range, so both read 0. The padding rows of U and of the
  // client's V block are 0 as well, hence R = 0 there and such entries add
  // nothing to S, Lambda or the statistics: no per-entry masks are needed.
  uint32_t vm[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = arow0 + 16 * rt + li;
      vm[rt][v] = row < p.m ? ((uint32_t)((4 * lg + v) * cl.ldm) + (uint32_t)row) * 4u : kOffNone;
    }

  // Operands of one 16-column chunk; a ring of kSDepth chunks is kept in
  // flight so that each wave has the next chunk's M loads outstanding while it
  // computes (vector loads complete in order, so everything a chunk needs is
  // issued together). Two measured faster than three, four or five at r = 20
  // and r = 40 (39 against 41, 49 and 52 us at 4000 x 8000, r = 20).
  // With two phases the halves of the work-group take alternate chunks; their
  // partial P are summed in LDS at the end.
  struct Chunk {
    float m[2][4];   // M[row][col] for this lane's rows (two 16-row tiles) and 4 columns
    float va[NS];    // MFMA 1 A operand (V A-packing): V[col j0 + l%16][rank (l/16)*NS + s]
    f4 vb[RTF > 0 ? RTF : 1];  // MFMA 2 B operand (V B-packing): V[col j0 + 4*(l/16) + e][rank 16*ct + l%16]
    f4 vq[NQ > 0 ? NQ : 1];    // quads: V[col j0 + 4*(l/16) + e][rank RP - 16 + 4 q + l%4]
  };
  constexpr int kSDepth = 2;
  Chunk ring[kSDepth];
  const int nch = (cl.n + 15) >> 4;
  const int nk = (nch - phase + NPH - 1) / NPH;  // chunks phase, phase + NPH, ... below nch
  auto load_chunk = [&](Chunk& c, int k) {
    const int j0 = (phase + NPH * k) << 4;
    const uint32_t vch = (uint32_t)((cl.vrow0 + j0) >> 4);
#pragma unroll
    for (int s = 0; s < NS; ++s) c.va[s] = bload(rVa, (uint32_t)lane * 4u, ((vch * NS + s) * 64u) * 4u);
#pragma unroll
    for (int ct = 0; ct < RTF; ++ct) c.vb[ct] = bload4(rVb, (uint32_t)lane * 16u, ((vch * RT + ct) * 64u) * 16u);
#pragma unroll
    for (int q = 0; q < NQ; ++q) c.vq[q] = bload4(rVq, vq_off, (vch * NQ + q) * 256u);
    const rsrc_t rM = make_rsrc(cl.M + (int64_t)j0 * cl.ldm, chunk_bytes_from(cl.n, j0, cl.ldm));
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) c.m[rt][v] = bload(rM, vm[rt][v], 0);
  };
  auto compute_chunk = [&](const Chunk& c, int k) {
    const int j0 = (phase + NPH * k) << 4;
    float l2 = 0.f, l1 = 0.f;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      f4 a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NS; ++s) a1 = mfma4(c.va[s], ub[rt][s], a1);
      f4 lamv;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float R = c.m[rt][v] - a1[v];
        const float L = __builtin_amdgcn_fmed3f(R, -lam, lam);  // clip(R, -lam, lam)
        const float Sv = R - L;
        if (STORE) {
          const int row = arow0 + 16 * rt + li, col = j0 + 4 * lg + v;
          if (row < p.m && col < cl.n) Sblk[(int64_t)col * lds_out + row] = Sv;
        }
        lamv[v] = L;
        l2 = fmaf(L, L, l2);
        l1 += fabsf(Sv);
        nnz += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(Sv != 0.f));
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int ct = 0; ct < RTF; ++ct) accp[rt][ct] = mfma4(lamv[s], c.vb[ct][s], accp[rt][ct]);
#pragma unroll
        for (int q = 0; q < NQ; ++q) accq[rt][q] = mfma4x4(lamv[s], c.vq[q][s], accq[rt][q]);
      }
    }
    sl2 += (double)l2;
    sl1 += (double)l1;
  };
  // Uniform loop: every iteration loads (chunk index clamped to the wave's
  // last chunk), so the wait counts stay exact; iterations past the wave's
  // chunks compute nothing (a wave-uniform branch).
  if (nk > 0) {
    const int nkp = (nk + kSDepth - 1) / kSDepth * kSDepth;
    // The prologue issues the ring in slot order (fenced like the loop body),
    // so that at the loop head slot 0 holds the oldest loads on every path.
#pragma unroll
    for (int d = 0; d < kSDepth; ++d) {
      load_chunk(ring[d], min(d, nk - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    if (!emit_only && closed) {
#pragma unroll
      for (int q = 0; q < kFabPer; ++q) {
        const int e = tid + q * 256 * NPH;
        if (e < RP * RP) {
          fab[0][e] = fa[q];
          fab[1][e] = fbv[q];
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    for (int k0 = 0; k0 < nkp; k0 += kSDepth) {
#pragma unroll
      for (int d = 0; d < kSDepth; ++d) {
        const int k = k0 + d;
        if (k < nk) compute_chunk(ring[d], k);
        // Keep the refill at this point of the program: left alone, the
        // scheduler sinks loads towards their first use and the ring
        // collapses to a single chunk in flight.
        __builtin_amdgcn_sched_barrier(0);
        load_chunk(ring[d], min(k + kSDepth, nk - 1));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else if (!emit_only && closed) {
    // A phase with no chunk (a client of at most 16 columns) still stages its
    // share of A_i and B_i.
#pragma unroll
    for (int q = 0; q < kFabPer; ++q) {
      const int e = tid + q * 256 * NPH;
      if (e < RP * RP) {
        fab[0][e] = fa[q];
        fab[1][e] = fbv[q];
      }
    }
  }

  if (emit_only) return;
  // Epilogue: the client's U-step term for these 128 rows. U_i comes from
  // the MFMA operand registers (rank (l/16) NS + s of row l%16; ranks from
  // 4 NS on are zero), P from the two phases' accumulators summed in LDS.
  // Quads: block b = l/4 summed columns 4 (b/4) + s for rows 4 (b%4) + i; the
  // four column groups (lanes l, l ^ 16, l ^ 32, l ^ 48) are added first.
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float x = accq[rt][q][i];
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        accq[rt][q][i] = x;
      }
  if (phase == 0) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
#pragma unroll
      for (int ct = 0; ct < RTF; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) ptile[w * 32 + 16 * rt + 4 * lg + v][16 * ct + li] = accp[rt][ct][v];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (lane < 16) ptile[w * 32 + 16 * rt + 4 * (lane >> 2) + i][16 * RTF + 4 * q + (lane & 3)] = accq[rt][q][i];
#pragma unroll
      for (int s = 0; s < NS; ++s) utile[w * 32 + 16 * rt + li][lg * NS + s] = ub[rt][s];
    }
  }
  if (phase == NPH - 1) {
    for (int c = 4 * NS + lg; c < RP; c += 4) {
      utile[w * 32 + li][c] = 0.f;
      utile[w * 32 + 16 + li][c] = 0.f;
    }
  }
  __syncthreads();
  if (NPH == 2 && phase == 1) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
#pragma unroll
      for (int ct = 0; ct < RTF; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) ptile[w * 32 + 16 * rt + 4 * lg + v][16 * ct + li] += accp[rt][ct][v];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (lane < 16) ptile[w * 32 + 16 * rt + 4 * (lane >> 2) + i][16 * RTF + 4 * q + (lane & 3)] += accq[rt][q][i];
    }
  }
  __syncthreads();
  spass_terms_and_stats<RP, 4 * NPH>(p, cl, b, ptile, utile, fab, closed, sl2, sl1, nnz);
}

// Partial Gram of kURows rows held in LDS (FP64, row stride kMaxRank), by a
// 256-thread work-group: thread (ta, tb) = (tid / 16, tid % 16) forms the
// RT x RT block of entries (RT ta + x, RT tb + y), so each LDS read feeds RT
// FMAs. Every entry is summed as two chains, even rows and odd rows, each in
// row order, then added.
template <int RT>
__device__ void gram_rows_partial(const double* ul, double* out) {
  constexpr int RP = 16 * RT;
  const int a0 = RT * (threadIdx.x >> 4), b0 = RT * (threadIdx.x & 15);
  double s0[RT][RT], s1[RT][RT];
#pragma unroll
  for (int x = 0; x < RT; ++x)
#pragma unroll
    for (int y = 0; y < RT; ++y) s0[x][y] = s1[x][y] = 0.0;
#pragma unroll 4
  for (int j = 0; j < kURows; j += 2) {
    double va0[RT], vb0[RT], va1[RT], vb1[RT];
#pragma unroll
    for (int x = 0; x < RT; ++x) {
      va0[x] = ul[j * kMaxRank + a0 + x];
      vb0[x] = ul[j * kMaxRank + b0 + x];
      va1[x] = ul[(j + 1) * kMaxRank + a0 + x];
      vb1[x] = ul[(j + 1) * kMaxRank + b0 + x];
    }
#pragma unroll
    for (int x = 0; x < RT; ++x)
#pragma unroll
      for (int y = 0; y < RT; ++y) {
        s0[x][y] += va0[x] * vb0[y];
        s1[x][y] += va1[x] * vb1[y];
      }
  }
#pragma unroll
  for (int x = 0; x < RT; ++x)
#pragma unroll
    for (int y = 0; y < RT; ++y) out[(a0 + x) * RP + b0 + y] = s0[x][y] + s1[x][y];
}

// ---------------------------------------------------------------------------
// U update. grid = (MP / 64, final ? 1 : E), 256 threads; thread (a = tid % 64,
// cq = tid / 64) owns row a and rank columns cq, cq + 4, ... The S-pass left
// each client's U-step term T_i in p.P.
// final = 1: U^(t+1) = mean_i T_i (eq. "U_agg") into the consensus buffer,
//            ||U^(t+1) - U^(t)||^2 partials and Gram slot 0;
// final = 0: U_i = T_i (intermediate local steps), Gram slot i.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_uupdate(DevParams p, float* __restrict__ Uout,
                                                 int64_t uout_stride,
                                                 const float* __restrict__ Uprev, int final_step) {
  constexpr int RP = 16 * RT, NQ = RP / 4;
  __shared__ double ul[kURows * kMaxRank];
  __shared__ double dred[4];
  const int MP = p.MP, r = p.r;
  const int tid = threadIdx.x, al = tid & 63, cq = tid >> 6;
  const int a = blockIdx.x * kURows + al;
  const int i_first = final_step ? 0 : (int)blockIdx.y;
  const int i_last = final_step ? p.E : (int)blockIdx.y + 1;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  // Clients are summed in order, kUB at a time so that their loads are in
  // flight together.
  constexpr int kUB = RT <= 2 ? 8 : 4;
  int i = i_first;
  for (; i + kUB <= i_last; i += kUB) {
    float tv[kUB][NQ];
#pragma unroll
    for (int u = 0; u < kUB; ++u) {
      const float* __restrict__ Ti = p.P + (int64_t)(i + u) * RP * MP + a;
#pragma unroll
      for (int q = 0; q < NQ; ++q) tv[u][q] = Ti[(int64_t)(cq + 4 * q) * MP];
    }
#pragma unroll
    for (int u = 0; u < kUB; ++u)
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] += (double)tv[u][q];
  }
  for (; i < i_last; ++i) {
    const float* __restrict__ Ti = p.P + (int64_t)i * RP * MP + a;
    float tv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) tv[q] = Ti[(int64_t)(cq + 4 * q) * MP];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += (double)tv[q];
  }
  // The previous consensus U (final step), loaded as one batch without a
  // branch (a load under a branch gets its own wait): other steps read a
  // valid stand-in and ignore it.
  float uprev[NQ];
  {
    const float* __restrict__ Upv = final_step ? Uprev : p.P;
#pragma unroll
    for (int q = 0; q < NQ; ++q) uprev[q] = Upv[(int64_t)(cq + 4 * q) * MP + a];
  }
  const double scale = final_step ? 1.0 / (double)p.E : 1.0;
  float* __restrict__ Uo = Uout + (final_step ? 0 : (int64_t)blockIdx.y * uout_stride);
  double dsq = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = cq + 4 * q;
    const float v = (a < p.m && c < r) ? (float)(acc[q] * scale) : 0.f;
    fb_store(Uo, MP, RP, p.NS, a, c, v);
    if (p.bf16) hb_store(u_hb(Uo, p), MP, p, a, c, v);
    ul[al * kMaxRank + c] = (double)v;
    if (final_step) {
      const double d = (double)v - (double)uprev[q];
      dsq += d * d;
    }
  }
  dsq = wave_sum(dsq);
  if ((tid & 63) == 0) dred[tid >> 6] = dsq;
  __syncthreads();
  const int slot = final_step ? 0 : (int)blockIdx.y;
  gram_rows_partial<RT>(ul, p.gram_part + ((int64_t)slot * p.nub + blockIdx.x) * RP * RP);
  if (final_step && tid == 0) p.upart[blockIdx.x] = dred[0] + dred[1] + dred[2] + dred[3];
}

// Gram partials of the consensus U (start of the run).
__global__ __launch_bounds__(256) void k_gram_init(DevParams p, const float* __restrict__ U) {
  __shared__ double ul[kURows * kMaxRank];
  const int RP = p.RP;
  for (int e = threadIdx.x; e < kURows * RP; e += blockDim.x) {
    const int al = e % kURows, c = e / kURows;
    ul[al * kMaxRank + c] = (double)U[(int64_t)c * p.MP + blockIdx.x * kURows + al];
  }
  __syncthreads();
  double* out = p.gram_part + (int64_t)blockIdx.x * RP * RP;
  switch (RP / 16) {
    case 1: gram_rows_partial<1>(ul, out); break;
    case 2: gram_rows_partial<2>(ul, out); break;
    case 3: gram_rows_partial<3>(ul, out); break;
    default: gram_rows_partial<4>(ul, out); break;
  }
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
__device__ void fin_gram(const DevParams& p, int gi, double* A) {
  const int r = p.r, RP = p.RP;
  const int64_t RR = (int64_t)RP * RP;
  const double* gp = p.gram_part + (int64_t)gi * p.nub * RR;
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    const int a = e / r, b = e - (e / r) * r;
    A[e] = sum_strided(gp + a * RP + b, p.nub, RR);
  }
}

// Round statistics from the partials of the round's kernels; result in
// out[0..5] of thread 0: ||Lambda||^2, ||S||_1, nnz(S), ||V||^2, ||dU||^2 and
// the U penalty of the objective at the round's start.
__device__ void fin_stats(const DevParams& p, double* out) {
  __shared__ double red[kFinThreads / 64][5];
  const int tid = threadIdx.x, r = p.r, RP = p.RP;
  const int64_t RR = (int64_t)RP * RP;
  if (tid < kFinThreads) {
    const int nsp = p.E * p.nrb;
    double l2 = block_strided_sum(nsp, [&](int k) { return p.spart[(int64_t)k * 4 + 0]; }, kFinThreads);
    double l1 = block_strided_sum(nsp, [&](int k) { return p.spart[(int64_t)k * 4 + 1]; }, kFinThreads);
    double nz = block_strided_sum(nsp, [&](int k) { return p.spart[(int64_t)k * 4 + 2]; }, kFinThreads);
    double vsq = block_strided_sum(p.ngroups * r, [&](int k) {
      const int g = k / r, d = k - g * r;
      return p.gv_part[(int64_t)g * RR + d * RP + d];
    }, kFinThreads);
    double du = block_strided_sum(p.nub, [&](int k) { return p.upart[k]; }, kFinThreads);
    l2 = wave_sum(l2);
    l1 = wave_sum(l1);
    nz = wave_sum(nz);
    vsq = wave_sum(vsq);
    du = wave_sum(du);
    if ((tid & 63) == 0) {
      red[tid >> 6][0] = l2;
      red[tid >> 6][1] = l1;
      red[tid >> 6][2] = nz;
      red[tid >> 6][3] = vsq;
      red[tid >> 6][4] = du;
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
  }
}

// G^{-1} of the Gram in LDS A (adds rho I) into Ginv slot gi; returns
// tr(U^T U) (valid in every thread).
__device__ double fin_inverse(const DevParams& p, double* A, double* Ginv, int64_t g_stride, int gi) {
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
  spd_inverse<kFinEPT>(A, r, r);
  double* Gout = Ginv + (int64_t)gi * g_stride;
  for (int e = tid; e < RR; e += blockDim.x) {
    const int a = e / RP, b = e % RP;
    Gout[e] = (a < r && b < r) ? A[a * r + b] : 0.0;
  }
  return tr_sh;
}

// Round record from the statistics and tr(U^(t+1)T U^(t+1)) (one thread).
__device__ void fin_record(const DevParams& p, const double* stats, double tr) {
  const int64_t t = p.dstate->t;
  StatsRec rec;
  rec.t = (double)t;
  rec.objective = 0.5 * stats[0] + 0.5 * p.rho * stats[3] + (double)p.lam_rec * stats[1] + stats[5];
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

// Standalone finalize: one work-group per Gram slot (grid = per_client ? E : 1).
__global__ __launch_bounds__(kFinThreads) void k_finalize(DevParams p, double* Ginv,
                                                          int64_t g_stride, int per_client,
                                                          int record) {
  __shared__ double A[kMaxRank * kMaxRank];
  __shared__ double st[6];
  const int gi = (int)blockIdx.x;
  fin_gram(p, gi, A);
  if (record && !per_client) fin_stats(p, st);
  __syncthreads();
  const double tr = fin_inverse(p, A, Ginv, g_stride, gi);
  if (threadIdx.x != 0) return;
  if (per_client)
    p.ucl_sq[gi] = tr;
  else if (!record)
    p.dstate->u_sq = tr;
  else
    fin_record(p, st, tr);
}

// The same work folded into a V-pass launch, by work-group role: role 0 forms
// the Gram and its inverse (into Ginv slot 0, trace into dstate->u_sq_next),
// role 1 the statistics (into p.stat_part). Neither reads what the other or
// the streaming work-groups write; the V finish records the round.
__device__ void finalize_role(const DevParams& p, double* Ginv, int role) {
  if (role == 0) {
    __shared__ double A[kMaxRank * kMaxRank];
    fin_gram(p, 0, A);
    __syncthreads();
    const double tr = fin_inverse(p, A, Ginv, 0, 0);
    if (threadIdx.x == 0) p.dstate->u_sq_next = tr;
  } else {
    __shared__ double st[6];
    fin_stats(p, st);
    if (threadIdx.x == 0)
      for (int q = 0; q < 6; ++q) p.stat_part[q] = st[q];
  }
}

// U^(0) into a factor block (zeros outside m x r).
__global__ void k_copy_in_U(DevParams p, const float* __restrict__ U0, int64_t ldu,
                            float* __restrict__ Ufb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)p.RP * p.MP) return;
  const int a = (int)(e % p.MP), c = (int)(e / p.MP);
  const float v = (a < p.m && c < p.r) ? U0[(int64_t)c * ldu + a] : 0.f;
  fb_store(Ufb, p.MP, p.RP, p.NS, a, c, v);
  if (p.bf16) hb_store(u_hb(Ufb, p), p.MP, p, a, c, v);
}

// L_i = U V_i^T (FP64 accumulation) and S_i, for one client, column-major out.
// grid.y strides over the client's columns.
__global__ void k_materialize(DevParams p, const float* __restrict__ Ucol, int client,
                              float* __restrict__ L, int64_t ldl, float* __restrict__ S,
                              int64_t lds_out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= p.m) return;
  const ClientDev cl = p.clients[client];
  for (int j = blockIdx.y; j < cl.n; j += gridDim.y) {
    if (L) {
      double s = 0.0;
      for (int c = 0; c < p.r; ++c)
        s += (double)Ucol[(int64_t)c * p.MP + a] *
             (double)p.V[(int64_t)(cl.vrow0 + j) * p.RP + c];
      L[(int64_t)j * ldl + a] = (float)s;
    }
    if (S) S[(int64_t)j * lds_out + a] = p.S[cl.s_off + (int64_t)j * p.lds + a];
  }
}

// Factors out: U (m x r) and V rows of one client (column-major, ld ldv).
__global__ void k_get_U(DevParams p, const float* __restrict__ Ucol, float* __restrict__ U,
                        int64_t ldu) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)p.m * p.r) return;
  const int a = (int)(e % p.m), c = (int)(e / p.m);
  U[(int64_t)c * ldu + a] = Ucol[(int64_t)c * p.MP + a];
}

__global__ void k_get_V(DevParams p, int client, int64_t col0, float* __restrict__ V, int64_t ldv) {
  const ClientDev cl = p.clients[client];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)cl.n * p.r) return;
  const int j = (int)(e % cl.n), c = (int)(e / cl.n);
  V[(int64_t)c * ldv + col0 + j] = p.V[(int64_t)(cl.vrow0 + j) * p.RP + c];
}

// Target factors into padded layouts: Ut column-major MP x RPT, Vt column-major
// NVP x RPT following the clients' padded V rows.
__global__ void k_pack_target_U(DevParams p, const float* __restrict__ Us, int64_t ldus, int rs,
                                float* __restrict__ Ut, int RPT) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)RPT * p.MP) return;
  const int a = (int)(e % p.MP), c = (int)(e / p.MP);
  Ut[e] = (a < p.m && c < rs) ? Us[(int64_t)c * ldus + a] : 0.f;
}

__global__ void k_pack_target_V(DevParams p, const float* __restrict__ Vs, int64_t ldvs, int rs,
                                float* __restrict__ Vt, int RPT, int client, int64_t col0) {
  const ClientDev cl = p.clients[client];
  const int span = (cl.n + kVPad - 1) / kVPad * kVPad;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)span * RPT) return;
  const int j = (int)(e % span), c = (int)(e / span);
  Vt[(int64_t)c * p.NVP + cl.vrow0 + j] = (j < cl.n && c < rs) ? Vs[(int64_t)c * ldvs + col0 + j] : 0.f;
}

// Partial cross-Gram matrices for ||X1 Y1^T - X2 Y2^T||_F^2. Work-groups
// [0, kDistBlocks) sweep the X side (MP rows), [kDistBlocks, 2 kDistBlocks) the
// Y side (NVP rows), 64 rows at a time. part[blk] holds [Z1^T Z1 | Z1^T Z2 |
// Z2^T Z2] as 64x64 FP64 tiles; each thread keeps 48 entries in registers.
constexpr int kDistRows = 64;
constexpr int kDistEntries = 3 * kMaxRank * kMaxRank;
__global__ __launch_bounds__(256) void k_dist_partial(DevParams p, const float* __restrict__ X1,
                                                      const float* __restrict__ Y1, int rp1,
                                                      const float* __restrict__ X2,
                                                      const float* __restrict__ Y2, int rp2,
                                                      double* __restrict__ part) {
  __shared__ float z1[kDistRows][kMaxRank + 1];
  __shared__ float z2[kDistRows][kMaxRank + 1];
  constexpr int kPer = kDistEntries / 256;
  const bool xside = (int)blockIdx.x < kDistBlocks;
  const int blk = xside ? blockIdx.x : blockIdx.x - kDistBlocks;
  const int ld = xside ? p.MP : p.NVP;
  const float* A = xside ? X1 : Y1;
  const float* B = xside ? X2 : Y2;
  double acc[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
  for (int row0 = blk * kDistRows; row0 < ld; row0 += kDistBlocks * kDistRows) {
    __syncthreads();
    for (int e = threadIdx.x; e < kDistRows * kMaxRank; e += blockDim.x) {
      const int j = e % kDistRows, c = e / kDistRows;
      const int row = row0 + j;
      z1[j][c] = (row < ld && c < rp1) ? A[(int64_t)c * ld + row] : 0.f;
      z2[j][c] = (row < ld && c < rp2) ? B[(int64_t)c * ld + row] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = threadIdx.x + q * 256;
      const int which = e / (kMaxRank * kMaxRank);
      const int a = (e / kMaxRank) % kMaxRank, b = e % kMaxRank;
      const int ra = which == 2 ? rp2 : rp1;
      const int rb = which == 0 ? rp1 : rp2;
      if (a < ra && b < rb) {
        const float(*za)[kMaxRank + 1] = which == 2 ? z2 : z1;
        const float(*zb)[kMaxRank + 1] = which == 0 ? z1 : z2;
        double s = 0.0;
        for (int j = 0; j < kDistRows; ++j) s += (double)za[j][a] * (double)zb[j][b];
        acc[q] += s;
      }
    }
  }
  double* o = part + (int64_t)blockIdx.x * kDistEntries;
#pragma unroll
  for (int q = 0; q < kPer; ++q) o[threadIdx.x + q * 256] = acc[q];
}

// Level 1: 48 work-groups x 256 entries; each entry's X- and Y-side Grams are
// summed over the partials and multiplied; part2[blk][which] = block sum.
__global__ __launch_bounds__(256) void k_dist_reduce(const double* __restrict__ part,
                                                     double* __restrict__ part2) {
  __shared__ double red[4];
  const int e = blockIdx.x * 256 + threadIdx.x;
  double gx = 0.0, gy = 0.0;
  for (int k = 0; k < kDistBlocks; ++k) gx += part[(int64_t)k * kDistEntries + e];
  for (int k = 0; k < kDistBlocks; ++k) gy += part[(int64_t)(kDistBlocks + k) * kDistEntries + e];
  double t = wave_sum(gx * gy);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) part2[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_dist_final(const double* __restrict__ part2, double* __restrict__ out2) {
  if (threadIdx.x != 0) return;
  constexpr int per = (kMaxRank * kMaxRank) / 256;  // level-1 blocks per Gram pair
  double s[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 3 * per; ++k) s[k / per] += part2[k];
  out2[0] = s[0] - 2.0 * s[1] + s[2];
  out2[1] = s[2];
}

// ---------------------------------------------------------------------------
// Launch helpers.
// ---------------------------------------------------------------------------
template <int RT, int NS>
static hipError_t launch_vpass_t(const DevParams& p, int mode, const float* U, int64_t u_stride,
                                 const float* Uold, const float* Vold, double* fin_Ginv,
                                 hipStream_t st) {
  const int fin = fin_Ginv ? 1 : 0;
  dim3 grid(p.ng64 * p.vsplit + (fin ? 2 : 0)), block(256);
  auto go = [&](auto kg) {
    constexpr int KG = decltype(kg)::value;
    if (mode == kSZero)
      hipLaunchKernelGGL((k_vpass<RT, NS, kSZero, KG>), grid, block, 0, st, p, U, u_stride, Uold,
                         Vold, fin_Ginv, fin);
    else if (mode == kSStored)
      hipLaunchKernelGGL((k_vpass<RT, NS, kSStored, KG>), grid, block, 0, st, p, U, u_stride,
                         Uold, Vold, fin_Ginv, fin);
    else
      hipLaunchKernelGGL((k_vpass<RT, NS, kSRecompute, KG>), grid, block, 0, st, p, U, u_stride,
                         Uold, Vold, fin_Ginv, fin);
  };
  if (p.vcols == 4)
    go(std::integral_constant<int, 4>{});
  else
    go(std::integral_constant<int, 1>{});
  return hipGetLastError();
}
template <int RT>
static hipError_t launch_vfinal_t(const DevParams& p, const double* Ginv, int64_t g_stride,
                                  int rec, hipStream_t st) {
  hipLaunchKernelGGL(k_vfinal<RT>, dim3(p.ngroups), dim3(256), 0, st, p, Ginv, g_stride, rec);
  return hipGetLastError();
}

template <int RT, int NS>
static hipError_t launch_spass_t(const DevParams& p, const float* U, int64_t u_stride, float* Sout,
                                 int64_t lds_out, int emit_only, int client_base,
                                 int client_count, hipStream_t st) {
  // Stored-S rounds and the rebuilt-S ones take the same column phases, so
  // both sum P in the same order.
  const dim3 grid(p.nrb, client_count);
  if (p.sphases == 1) {
    if (Sout)
      hipLaunchKernelGGL((k_spass<RT, NS, true, 1>), grid, dim3(256), 0, st, p, U, u_stride, Sout,
                         lds_out, emit_only, client_base);
    else
      hipLaunchKernelGGL((k_spass<RT, NS, false, 1>), grid, dim3(256), 0, st, p, U, u_stride, Sout,
                         lds_out, emit_only, client_base);
  } else {
    if (Sout)
      hipLaunchKernelGGL((k_spass<RT, NS, true, 2>), grid, dim3(512), 0, st, p, U, u_stride, Sout,
                         lds_out, emit_only, client_base);
    else
      hipLaunchKernelGGL((k_spass<RT, NS, false, 2>), grid, dim3(512), 0, st, p, U, u_stride, Sout,
                         lds_out, emit_only, client_base);
  }
  return hipGetLastError();
}

// Compile-time (RT, NS) dispatch: NS = ceil(r/4) lies in [4 RT - 3, 4 RT].
template <int RT, int NS, class F>
static hipError_t with_ns(int ns, F&& f) {
  if (ns == NS) return f(std::integral_constant<int, RT>{}, std::integral_constant<int, NS>{});
  if constexpr (NS < 4 * RT) return with_ns<RT, NS + 1>(ns, f);
  return hipErrorInvalidValue;
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

hipError_t launch_vpass(const DevParams& p, int mode, const float* U, int64_t u_stride,
                        const float* Uold, const float* Vold, double* fin_Ginv, hipStream_t st) {
  return with_rank(p, [&](auto rt, auto ns) {
    return launch_vpass_t<decltype(rt)::value, decltype(ns)::value>(p, mode, U, u_stride, Uold,
                                                                   Vold, fin_Ginv, st);
  });
}

hipError_t launch_vfinal(const DevParams& p, const double* Ginv, int64_t g_stride, int rec,
                         hipStream_t st) {
  return with_rank(p, [&](auto rt, auto) {
    return launch_vfinal_t<decltype(rt)::value>(p, Ginv, g_stride, rec, st);
  });
}

hipError_t launch_client_factor(const DevParams& p, hipStream_t st) {
  hipLaunchKernelGGL(k_client_factor, dim3(p.E), dim3(1024), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_spass(const DevParams& p, const float* U, int64_t u_stride, float* Sout,
                        int64_t lds_out, int emit_only, int client_base, int client_count,
                        hipStream_t st) {
  return with_rank(p, [&](auto rt, auto ns) {
    return launch_spass_t<decltype(rt)::value, decltype(ns)::value>(
        p, U, u_stride, Sout, lds_out, emit_only, client_base, client_count, st);
  });
}

hipError_t launch_uupdate(const DevParams& p, float* Uout, int64_t uout_stride,
                          const float* Uprev_cons, int final_step, hipStream_t st) {
  dim3 grid(p.nub, final_step ? 1 : p.E), block(256);
  switch (p.RP / 16) {
    case 1: hipLaunchKernelGGL(k_uupdate<1>, grid, block, 0, st, p, Uout, uout_stride, Uprev_cons, final_step); break;
    case 2: hipLaunchKernelGGL(k_uupdate<2>, grid, block, 0, st, p, Uout, uout_stride, Uprev_cons, final_step); break;
    case 3: hipLaunchKernelGGL(k_uupdate<3>, grid, block, 0, st, p, Uout, uout_stride, Uprev_cons, final_step); break;
    case 4: hipLaunchKernelGGL(k_uupdate<4>, grid, block, 0, st, p, Uout, uout_stride, Uprev_cons, final_step); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const DevParams& p, double* Ginv, int64_t g_stride, int per_client,
                           int record, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(per_client ? p.E : 1), dim3(kFinThreads), 0, st, p, Ginv,
                     g_stride, per_client, record);
  return hipGetLastError();
}

hipError_t launch_gram_init(const DevParams& p, const float* U, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_init, dim3(p.nub), dim3(256), 0, st, p, U);
  return hipGetLastError();
}

hipError_t launch_copy_in_U(const DevParams& p, const float* U0, int64_t ldu, float* Ufb,
                            hipStream_t st) {
  const int64_t tot = (int64_t)p.RP * p.MP;
  hipLaunchKernelGGL(k_copy_in_U, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p, U0,
                     ldu, Ufb);
  return hipGetLastError();
}

hipError_t launch_materialize(const DevParams& p, const ClientDev* host_clients,
                              const int64_t* col_off, const float* Ucol, int client_begin,
                              int client_end, float* L, int64_t ldl, float* S, int64_t lds,
                              hipStream_t st) {
  for (int i = client_begin; i < client_end; ++i) {
    const int64_t c0 = col_off[i] - col_off[client_begin];
    const int ny = host_clients[i].n < 65535 ? host_clients[i].n : 65535;
    dim3 grid((unsigned)((p.m + 255) / 256), (unsigned)ny);
    hipLaunchKernelGGL(k_materialize, grid, dim3(256), 0, st, p, Ucol, i,
                       L ? L + c0 * ldl : nullptr, ldl, S ? S + c0 * lds : nullptr, lds);
  }
  return hipGetLastError();
}

hipError_t launch_get_factors(const DevParams& p, const ClientDev* host_clients,
                              const int64_t* col_off, const float* Ucol, float* U, int64_t ldu,
                              float* V, int64_t ldv, hipStream_t st) {
  if (U) {
    const int64_t tot = (int64_t)p.m * p.r;
    hipLaunchKernelGGL(k_get_U, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p, Ucol,
                       U, ldu);
  }
  if (V) {
    for (int i = 0; i < p.E; ++i) {
      const int64_t tot = (int64_t)host_clients[i].n * p.r;
      hipLaunchKernelGGL(k_get_V, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p, i,
                         col_off[i], V, ldv);
    }
  }
  return hipGetLastError();
}

hipError_t launch_pack_target(const DevParams& p, const ClientDev* host_clients,
                              const int64_t* col_off, const float* Us, int64_t ldus,
                              const float* Vs, int64_t ldvs, int rs, float* Ut, float* Vt,
                              int RPT, hipStream_t st) {
  const int64_t totu = (int64_t)RPT * p.MP;
  hipLaunchKernelGGL(k_pack_target_U, dim3((unsigned)((totu + 255) / 256)), dim3(256), 0, st, p,
                     Us, ldus, rs, Ut, RPT);
  for (int i = 0; i < p.E; ++i) {
    const int span = (host_clients[i].n + kVPad - 1) / kVPad * kVPad;
    const int64_t tot = (int64_t)span * RPT;
    hipLaunchKernelGGL(k_pack_target_V, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       p, Vs, ldvs, rs, Vt, RPT, i, col_off[i]);
  }
  return hipGetLastError();
}

hipError_t launch_factor_distance(const DevParams& p, const float* X1, const float* Y1, int rp1,
                                  const float* X2, const float* Y2, int rp2, double* part,
                                  double* part2, double* out2, hipStream_t st) {
  hipLaunchKernelGGL(k_dist_partial, dim3(2 * kDistBlocks), dim3(256), 0, st, p, X1, Y1, rp1, X2,
                     Y2, rp2, part);
  hipLaunchKernelGGL(k_dist_reduce, dim3(kDistEntries / 256), dim3(256), 0, st, part, part2);
  hipLaunchKernelGGL(k_dist_final, dim3(1), dim3(64), 0, st, part2, out2);
  return hipGetLastError();
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

// The two BF16 copies of M (layouts in rpca_internal.h); grid = (blocks,
// clients), each thread forms 16-byte units of both layouts, zero outside
// the client's m x n_i block.
__global__ __launch_bounds__(256) void k_m_to_bf16(DevParams p) {
  const ClientDev cl = p.clients[blockIdx.y];
  const int MP = p.MP, m = p.m;
  const int nvc = (cl.n + kVPad - 1) / kVPad * kVPad;
  const int64_t units = (int64_t)nvc * MP / 8;
  const int64_t base = (int64_t)cl.vrow0 * MP;
  const GLOBAL float* M = gptr(cl.M);
  bf8* Mv = reinterpret_cast<bf8*>(p.Mbv + base);
  bf8* Ms = reinterpret_cast<bf8*>(p.Mbs + base);
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(u & 63), g = l >> 4, li = l & 15;
    const int64_t tile = u >> 6;
    float x[8];
    {
      const int ch = (int)(tile % (MP >> 5)), cg = (int)(tile / (MP >> 5));
      const int j = 16 * cg + li, a0 = 32 * ch + 8 * g;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        x[e] = (a0 + e < m && j < cl.n) ? M[(int64_t)j * cl.ldm + a0 + e] : 0.f;
      Mv[u] = pack8(x);
    }
    {
      const int cc = (int)(tile % (nvc >> 5)), rt = (int)(tile / (nvc >> 5));
      const int a = 16 * rt + li, j0 = 32 * cc + 8 * g;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        x[e] = (a < m && j0 + e < cl.n) ? M[(int64_t)(j0 + e) * cl.ldm + a] : 0.f;
      Ms[u] = pack8(x);
    }
  }
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

// ---------------------------------------------------------------------------
// BF16 V-pass, streaming part: same grid, work-group roles and output
// (W = (M_i - S_i)^T U partials per row split) as k_vpass. Every BF16
// operand of a 32-row chunk is a 1 KiB wave load, and the U operands of a
// chunk (hP halves for the S rebuild, hB for W) cost as many loads as M
// itself, so a wave takes KG 16-column groups of the tile, which share the
// chunk's U operands in registers, and the KG waves on the same columns split
// the rows (phase q takes chunks q, q + KG, ...); their partial W are added
// in LDS in phase order at the end.
// Lane l holds rows 8 (l/16) + e of column 16 g + l%16: the A operand of W's
// MFMA, with U's hB packing as B; accumulator W[col 16 g + 4 (l/16) + v]
// [rank 16 ct + l%16]. kSRecompute rebuilds S = soft(M - Uo Vo^T): two 16x16
// products per chunk and column group with the previous U's hP packing on the
// A side and the previous V's hA packing on the B side leave lane l the same
// eight rows of its column.
// X3 = false: M from the V-pass BF16 copy (one 16-byte load per lane), one
// BF16 product per contraction, KG = 4.
// X3 = true: M in FP32 from the caller's block (two 16-byte loads per lane),
// every product as three BF16 products of hi/lo splits (mfma3), KG = 2.
// ---------------------------------------------------------------------------
template <int RT, int NK, int MODE, bool X3>
__global__ __launch_bounds__(256) void k_vpass_h(DevParams p, const float* __restrict__ Ubase,
                                                 const float* __restrict__ Uold,
                                                 const float* __restrict__ Vold,
                                                 double* __restrict__ fin_Ginv, int fin) {
  constexpr int RP = 16 * RT;
  constexpr int KG = X3 ? 2 : 4, kPh = KG;  // column groups per wave, row phases
  int bid = (int)blockIdx.x;
  if (fin) {
    if (bid < 2) {
      finalize_role(p, fin_Ginv, bid);
      return;
    }
    bid -= 2;
  }
  const int gx = bid % p.ng64, gy = bid / p.ng64;
  const VTile vt = p.vg64[gx];
  const ClientDev& cl = vt.cl;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cset = w % (4 / kPh), ph = w / (4 / kPh);  // column set, row phase
  const int jw = vt.j0 + 16 * KG * cset;               // first column of this wave
  const float lam = p.lam;
  const int MP = p.MP;

  // Hi packings, and (X3) the lo packings one packing block further.
  const int64_t uhl = hb_elems(MP, p.RK, p.RP) / 8, vhl = hb_elems(p.NVP, p.RK, p.RP) / 8;
  const GLOBAL bf8* UhB = reinterpret_cast<const GLOBAL bf8*>(gptr(u_hb(Ubase, p))) +
                          2 * (int64_t)MP * p.RK / 8;
  const GLOBAL bf8* UohP = reinterpret_cast<const GLOBAL bf8*>(gptr(u_hb(Uold, p))) +
                           (int64_t)MP * p.RK / 8;
  bf8 vb[KG][NK], vbl[X3 ? KG : 1][NK];  // S rebuild B operand (hi, lo): Vo[col][rank 32 kb + 8 (l/16) + e]
  if (MODE == kSRecompute) {
    const GLOBAL bf8* VohA = reinterpret_cast<const GLOBAL bf8*>(gptr(v_hb(Vold, p)));
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const int vch = (cl.vrow0 + jw + 16 * g) >> 4;
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        vb[g][kb] = VohA[((int64_t)vch * NK + kb) * 64 + lane];
        if constexpr (X3) vbl[g][kb] = VohA[vhl + ((int64_t)vch * NK + kb) * 64 + lane];
      }
    }
  }
  const int rbeg = gy * p.vsplit_rows;
  const int rend = min(p.m, rbeg + p.vsplit_rows);
  const int ch0 = rbeg >> 5;
  const int nch = (rend - rbeg + 31) >> 5;
  const int nk = (nch - ph + kPh - 1) / kPh;  // this wave's chunks ph, ph + kPh, ...
  // M: the BF16 copy (column group cg = (jw + 16 g) / 16), or (X3) the
  // caller's FP32 block through one buffer resource per column group
  // (columns past n_i read 0; rows past m are masked in the last chunk).
  const GLOBAL u4* Mv = reinterpret_cast<const GLOBAL u4*>(gptr(p.Mbv)) +
                        (int64_t)cl.vrow0 * MP / 8 + (int64_t)(jw >> 4) * (MP >> 5) * 64 + lane;
  const int64_t gstride = (int64_t)(MP >> 5) * 64;  // u4 units between column groups
  rsrc_t rM[X3 ? KG : 1];
  uint32_t vM = 0;
  if constexpr (X3) {
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const int j0 = jw + 16 * g;
      rM[g] = make_rsrc(cl.M + (int64_t)min(j0, cl.n) * cl.ldm, block_bytes_from(cl.n, j0, cl.ldm));
    }
    vM = (uint32_t)(li * cl.ldm) * 4u;
  }
  f4 acc[KG][RT];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) acc[g][ct] = f4{0.f, 0.f, 0.f, 0.f};

  struct Chunk {
    u4 m[KG];                    // BF16 copy: M rows 32 ch + 8 (l/16) + e of column 16 g + l%16
    f4 mf[X3 ? KG : 1][2];       // X3: the same rows in FP32
    bf8 uo[2][NK], uol[X3 ? 2 : 1][NK];  // previous U, hP halves (hi, lo)
    bf8 u[RT], ul[X3 ? RT : 1];          // U, hB (hi, lo)
  };
  constexpr int kDepth = 2;
  Chunk ring[kDepth];
  auto load_chunk = [&](Chunk& c, int k) {
    const int ch = ch0 + ph + kPh * k;
    if constexpr (X3) {
      const uint32_t rowb = (uint32_t)(32 * ch + 8 * lg) * 4u;
#pragma unroll
      for (int g = 0; g < KG; ++g) {
        c.mf[g][0] = bload4(rM[g], vM + rowb, 0);
        c.mf[g][1] = bload4(rM[g], vM + rowb + 16u, 0);
      }
    } else {
#pragma unroll
      for (int g = 0; g < KG; ++g) c.m[g] = Mv[g * gstride + (int64_t)ch * 64];
    }
    if (MODE == kSRecompute) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
          const int64_t o = (((int64_t)ch * 2 + t) * NK + kb) * 64 + lane;
          c.uo[t][kb] = UohP[o];
          if constexpr (X3) c.uol[t][kb] = UohP[uhl + o];
        }
    }
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) {
      const int64_t o = ((int64_t)ch * RT + ct) * 64 + lane;
      c.u[ct] = UhB[o];
      if constexpr (X3) c.ul[ct] = UhB[uhl + o];
    }
  };
  auto compute_chunk = [&](const Chunk& c, int k) {
    // Rows past m and columns past n_i are zero in the BF16 copy and in the
    // factors' packings, so they give d = 0 without a mask; the FP32 block
    // holds the caller's rows past m, which are masked.
    const int row0 = 32 * (ch0 + ph + kPh * k) + 8 * lg;
    const bool tail = 32 * (ch0 + ph + kPh * k) + 32 > p.m;  // wave-uniform
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      float x[8], d[8];
      if constexpr (X3) {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = c.mf[g][e >> 2][e & 3];
        if (tail) {
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = row0 + e < p.m ? x[e] : 0.f;
        }
      } else {
        unpack8(c.m[g], x);
      }
      if (MODE == kSRecompute) {
        f4 o[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            if constexpr (X3)
              o[t] = mfma3(c.uo[t][kb], c.uol[t][kb], vb[g][kb], vbl[g][kb], o[t]);
            else
              o[t] = mfma_bf16(c.uo[t][kb], vb[g][kb], o[t]);
          }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float a1 = o[e >> 2][e & 3];
          // M - S = Uo Vo^T + clip(M - Uo Vo^T, -lambda, lambda)
          d[e] = a1 + __builtin_amdgcn_fmed3f(x[e] - a1, -lam, lam);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) d[e] = x[e];
      }
      if constexpr (X3) {
        bf8 dh, dl;
        split8(d, dh, dl);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) acc[g][ct] = mfma3(dh, dl, c.u[ct], c.ul[ct], acc[g][ct]);
      } else {
        const bf8 dh = pack8(d);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) acc[g][ct] = mfma_bf16(dh, c.u[ct], acc[g][ct]);
      }
    }
  };
  if (nk > 0) {
    // Uniform ring as in k_vpass: every iteration loads (index clamped to the
    // wave's last chunk), so the wait counts stay exact.
    const int nkp = (nk + kDepth - 1) / kDepth * kDepth;
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      load_chunk(ring[d], min(d, nk - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int k0 = 0; k0 < nkp; k0 += kDepth) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
        const int k = k0 + d;
        if (k < nk) compute_chunk(ring[d], k);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk(ring[d], min(k + kDepth, nk - 1));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // Partial W of the waves, added in LDS in row-phase order; the work-group
  // then writes its partial of the 64 columns.
  __shared__ float red[kVStreamCols][RP];
  const int c0 = 16 * KG * cset;
  for (int q0 = 0; q0 < kPh; ++q0) {
    if (ph == q0) {
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int ct = 0; ct < RT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float& x = red[c0 + 16 * g + 4 * lg + v][16 * ct + li];
            x = q0 == 0 ? acc[g][ct][v] : x + acc[g][ct][v];
          }
    }
    __syncthreads();
  }
  GLOBAL float* wp = gptr_w(p.Wpart) + ((int64_t)gy * p.NVP + cl.vrow0 + vt.j0) * RP;
  for (int e = tid; e < kVStreamCols * RP; e += blockDim.x) wp[e] = red[e / RP][e % RP];
}

// ---------------------------------------------------------------------------
// BF16 S-pass: same grid (128-row blocks x clients, widest client first) and
// outputs as k_spass, over 32-column chunks, with 256 threads. Each wave
// takes kRT 16-row tiles, which share each chunk's V operands in registers,
// and every (4 / kPh)-th chunk of its row group: X3 = false, four tiles and
// two column phases; X3 = true, two tiles and one phase. MFMA 1 forms
// (U V^T)^T for two 16x16 tiles per row tile with V's hP halves as A and U's
// hA as B, leaving lane l row l%16 and the eight columns 8 (l/16) + e of the
// chunk -- the lane's 16-byte load of the S-pass copy of M (X3: eight FP32
// loads from the caller's block), and the A operand of MFMA 2 (P += Lambda V
// with V's hB packing as B; X3: every product as three BF16 products of
// hi/lo splits). The phases' partial P are added in LDS in phase order. LDS
// holds P and FP32 copies of A_i and B_i (74 KB at r = 64), so two
// work-groups fit on a compute unit and one's epilogue overlaps the other's
// sweep.
// ---------------------------------------------------------------------------
template <int RT, int NK, bool X3>
__global__ __launch_bounds__(256) void k_spass_h(DevParams p, const float* __restrict__ U) {
  constexpr int RP = 16 * RT;
  constexpr int kRT = X3 ? 2 : 4;   // 16-row tiles per wave
  constexpr int kPh = X3 ? 1 : 2;   // column phases
  constexpr int kRG = 4 / kPh;      // row groups of 16 kRT rows
  static_assert(kRG * 16 * kRT == kSRows, "row groups cover the work-group's rows");
  const int b = blockIdx.x;
  const ClientDev cl = p.clients_lpt[blockIdx.y];
  const int ci = cl.idx;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rg = wv % kRG, phase = wv / kRG;
  const int li = lane & 15, lg = lane >> 4;
  const int arow0 = b * kSRows + rg * 16 * kRT;
  const int MP = p.MP;

  const int64_t uhl = hb_elems(MP, p.RK, p.RP) / 8, vhl = hb_elems(p.NVP, p.RK, p.RP) / 8;
  bf8 ub[kRT][NK], ubl[X3 ? kRT : 1][NK];  // MFMA 1 B operand (hi, lo): U[row][rank 32 kb + 8 (l/16) + e]
  {
    const GLOBAL bf8* UhA = reinterpret_cast<const GLOBAL bf8*>(gptr(u_hb(U, p)));
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        const int64_t o = ((int64_t)((arow0 >> 4) + rt) * NK + kb) * 64 + lane;
        ub[rt][kb] = UhA[o];
        if constexpr (X3) ubl[rt][kb] = UhA[uhl + o];
      }
  }
  f4 accp[kRT][RT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) accp[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};

  // A_i and B_i of the closed-form step, rounded to FP32, for the epilogue
  // (made visible by the barriers that add the phases' P). Rows are padded to
  // RP + 16 floats, so that the epilogue's operand reads (four rows of 16
  // consecutive entries per wave) fall in distinct banks.
  constexpr int kFS = RP + 16;
  __shared__ float fab[2][RP * kFS];
  const bool closed = p.u_mode != 0;
  if (closed) {
    const double* __restrict__ Af = p.Afac + (int64_t)ci * RP * RP;
    const double* __restrict__ Bf = p.Bfac + (int64_t)ci * RP * RP;
    for (int e = tid; e < RP * RP; e += blockDim.x) {
      const int at = (e / RP) * kFS + e % RP;
      fab[0][at] = (float)Af[e];
      fab[1][at] = (float)Bf[e];
    }
  }

  double sl2 = 0.0, sl1 = 0.0;
  uint32_t nnz = 0;
  const float lam = p.lam;
  const GLOBAL bf8* Vh = reinterpret_cast<const GLOBAL bf8*>(gptr(v_hb(p.V, p)));
  const GLOBAL bf8* VhP = Vh + (int64_t)p.NVP * p.RK / 8;
  const GLOBAL bf8* VhB = Vh + 2 * (int64_t)p.NVP * p.RK / 8;
  const int nvc32 = (cl.n + kVPad - 1) / kVPad * (kVPad / 32);
  const GLOBAL u4* Ms = reinterpret_cast<const GLOBAL u4*>(gptr(p.Mbs)) +
                        (int64_t)cl.vrow0 * MP / 8 + (int64_t)(arow0 >> 4) * nvc32 * 64 + lane;
  // X3: the caller's FP32 block, one buffer resource per chunk (base at its
  // first column), fixed per-lane offsets; columns past n_i are out of range
  // and rows past m get an offset beyond any range, so both read 0.
  uint32_t vm[X3 ? kRT : 1][8];
  if constexpr (X3) {
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      const int row = arow0 + 16 * rt + li;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        vm[rt][e] = row < p.m ? ((uint32_t)((8 * lg + e) * cl.ldm) + (uint32_t)row) * 4u : kOffNone;
    }
  }
  struct Chunk {
    u4 m[kRT];                  // M[row arow0 + 16 rt + l%16][col 32 cc + 8 (l/16) + e]
    float mf[X3 ? kRT : 1][8];  // X3: the same entries in FP32
    bf8 va[2][NK], val[X3 ? 2 : 1][NK];  // V hP halves (hi, lo)
    bf8 vb[RT], vbl[X3 ? RT : 1];        // V hB (hi, lo)
  };
  constexpr int kDepth = 2;
  Chunk ring[kDepth];
  const int nch = (cl.n + 31) >> 5;
  const int nk = (nch - phase + kPh - 1) / kPh;  // chunks phase, phase + kPh, ... below nch
  auto load_chunk = [&](Chunk& c, int k) {
    const int cc = phase + kPh * k;
    const int64_t vch = (cl.vrow0 >> 5) + cc;
    if constexpr (X3) {
      const rsrc_t rM = make_rsrc(cl.M + (int64_t)32 * cc * cl.ldm, chunk_bytes_from(cl.n, 32 * cc, cl.ldm));
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
        for (int e = 0; e < 8; ++e) c.mf[rt][e] = bload(rM, vm[rt][e], 0);
    } else {
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt) c.m[rt] = Ms[((int64_t)rt * nvc32 + cc) * 64];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        const int64_t o = ((vch * 2 + t) * NK + kb) * 64 + lane;
        c.va[t][kb] = VhP[o];
        if constexpr (X3) c.val[t][kb] = VhP[vhl + o];
      }
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) {
      const int64_t o = (vch * RT + ct) * 64 + lane;
      c.vb[ct] = VhB[o];
      if constexpr (X3) c.vbl[ct] = VhB[vhl + o];
    }
  };
  auto compute_chunk = [&](const Chunk& c) {
    float l2 = 0.f, l1 = 0.f;
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      f4 o[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if constexpr (X3)
            o[t] = mfma3(c.va[t][kb], c.val[t][kb], ub[rt][kb], ubl[rt][kb], o[t]);
          else
            o[t] = mfma_bf16(c.va[t][kb], ub[rt][kb], o[t]);
        }
      }
      float x[8], lamv[8];
      if constexpr (X3) {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = c.mf[rt][e];
      } else {
        unpack8(c.m[rt], x);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float R = x[e] - o[e >> 2][e & 3];
        const float L = __builtin_amdgcn_fmed3f(R, -lam, lam);  // clip(R, -lam, lam)
        const float Sv = R - L;
        lamv[e] = L;
        l2 = fmaf(L, L, l2);
        l1 += fabsf(Sv);
        nnz += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(Sv != 0.f));
      }
      if constexpr (X3) {
        bf8 lh, ll;
        split8(lamv, lh, ll);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) accp[rt][ct] = mfma3(lh, ll, c.vb[ct], c.vbl[ct], accp[rt][ct]);
      } else {
        const bf8 lh = pack8(lamv);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) accp[rt][ct] = mfma_bf16(lh, c.vb[ct], accp[rt][ct]);
      }
    }
    sl2 += (double)l2;
    sl1 += (double)l1;
  };
  if (nk > 0) {
    const int nkp = (nk + kDepth - 1) / kDepth * kDepth;
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      load_chunk(ring[d], min(d, nk - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int k0 = 0; k0 < nkp; k0 += kDepth) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
        const int k = k0 + d;
        if (k < nk) compute_chunk(ring[d]);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk(ring[d], min(k + kDepth, nk - 1));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  // P of the phases, added in LDS in phase order.
  __shared__ float ptile[kSRows][RP + 1];
  for (int q = 0; q < kPh; ++q) {
    if (phase == q) {
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
        for (int ct = 0; ct < RT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float& x = ptile[rg * 16 * kRT + 16 * rt + 4 * lg + v][16 * ct + li];
            x = q == 0 ? accp[rt][ct][v] : x + accp[rt][ct][v];
          }
    }
    __syncthreads();
  }
  // U-step term of these 128 rows, as in the FP32 form's epilogue but in
  // FP32 (the BF16 rounds' operands carry 8-bit significands, so FP32 here
  // adds nothing measurable).
  const int row0 = b * kSRows;
  float* Ti = p.P + (int64_t)ci * RP * p.MP;
  if (closed) {
    // T_i = P A_i + U_i B_i on FP32 MFMA, as its transpose A_i^T P^T +
    // B_i^T U_i^T in 16-rank x 16-row tiles: wave wv takes rows 32 wv .. +31
    // of the block, and lane l ends with T[row l%16][rank 4 (l/16) + v] of a
    // tile, so each store covers 16 consecutive rows of a rank column. P comes
    // from LDS, U_i (FP32) from its column-major layout.
    constexpr int kK = RP / 4;
    const int rb = 32 * wv;
    float ua[2][kK];  // U[row0 + rb + 16 rt + l%16][4 kk + l/16]
    {
      const GLOBAL float* Uc = gptr(U) + row0 + rb + li;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int kk = 0; kk < kK; ++kk) ua[rt][kk] = Uc[(int64_t)(4 * kk + lg) * MP + 16 * rt];
    }
    f4 acc[2][RT];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < RT; ++ct) acc[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int kk = 0; kk < kK; ++kk) {
      float pb[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) pb[rt] = ptile[rb + 16 * rt + li][4 * kk + lg];
#pragma unroll
      for (int ct = 0; ct < RT; ++ct) {
        const float a0 = fab[0][(4 * kk + lg) * kFS + 16 * ct + li];
        const float a1 = fab[1][(4 * kk + lg) * kFS + 16 * ct + li];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          acc[rt][ct] = mfma4(a0, pb[rt], acc[rt][ct]);
          acc[rt][ct] = mfma4(a1, ua[rt][kk], acc[rt][ct]);
        }
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < RT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * ct + 4 * lg + v;
          Ti[(int64_t)c * MP + row0 + rb + 16 * rt + li] = c < p.r ? acc[rt][ct][v] : 0.f;
        }
  } else {
    // Gradient step: thread tid owns row tid % 128 and the rank columns
    // 8 (tid / 128) + 16 q .. + 7.
    const int rl = tid & (kSRows - 1);
    const float eta = (float)eta_of_round(p, p.dstate->t);
    const float cc = (float)cl.c;
    for (int c0 = 8 * (tid >> 7); c0 < RP; c0 += 16) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float u = gptr(U)[(int64_t)(c0 + j) * MP + row0 + rl];
        const float t = u - eta * (cc * u - ptile[rl][c0 + j]);
        Ti[(int64_t)(c0 + j) * MP + row0 + rl] = c0 + j < p.r ? t : 0.f;
      }
    }
  }
  spass_stats<4>(p, ci, b, sl2, sl1, nnz);
}

hipError_t launch_m_to_bf16(const DevParams& p, hipStream_t st) {
  hipLaunchKernelGGL(k_m_to_bf16, dim3(1024, p.E), dim3(256), 0, st, p);
  return hipGetLastError();
}

// The contraction-side block count follows from the rank tiles:
// NK = ceil(r/32) = ceil(RT/2).
template <int RT>
static hipError_t launch_vpass_h_t(const DevParams& p, int mode, const float* U, const float* Uold,
                                   const float* Vold, double* fin_Ginv, int x3, hipStream_t st) {
  constexpr int NK = (RT + 1) / 2;
  const int fin = fin_Ginv ? 1 : 0;
  const dim3 grid((unsigned)(p.ng64 * p.vsplit + 2 * fin));
  auto go = [&](auto m, auto x) {
    hipLaunchKernelGGL((k_vpass_h<RT, NK, decltype(m)::value, decltype(x)::value>), grid,
                       dim3(256), 0, st, p, U, Uold, Vold, fin_Ginv, fin);
  };
  using Z = std::integral_constant<int, kSZero>;
  using R = std::integral_constant<int, kSRecompute>;
  using F = std::false_type;
  using T = std::true_type;
  if (mode == kSRecompute)
    x3 ? go(R{}, T{}) : go(R{}, F{});
  else
    x3 ? go(Z{}, T{}) : go(Z{}, F{});
  return hipGetLastError();
}

hipError_t launch_vpass_h(const DevParams& p, int mode, const float* U, const float* Uold,
                          const float* Vold, double* fin_Ginv, int x3, hipStream_t st) {
  if (mode != kSZero && mode != kSRecompute) return hipErrorInvalidValue;
  switch (p.RP / 16) {
    case 1: return launch_vpass_h_t<1>(p, mode, U, Uold, Vold, fin_Ginv, x3, st);
    case 2: return launch_vpass_h_t<2>(p, mode, U, Uold, Vold, fin_Ginv, x3, st);
    case 3: return launch_vpass_h_t<3>(p, mode, U, Uold, Vold, fin_Ginv, x3, st);
    case 4: return launch_vpass_h_t<4>(p, mode, U, Uold, Vold, fin_Ginv, x3, st);
    default: return hipErrorInvalidValue;
  }
}

template <int RT>
static hipError_t launch_spass_h_t(const DevParams& p, const float* U, int x3, hipStream_t st) {
  constexpr int NK = (RT + 1) / 2;
  const dim3 grid(p.nrb, p.E);
  if (x3)
    hipLaunchKernelGGL((k_spass_h<RT, NK, true>), grid, dim3(256), 0, st, p, U);
  else
    hipLaunchKernelGGL((k_spass_h<RT, NK, false>), grid, dim3(256), 0, st, p, U);
  return hipGetLastError();
}

hipError_t launch_spass_h(const DevParams& p, const float* U, int x3, hipStream_t st) {
  switch (p.RP / 16) {
    case 1: return launch_spass_h_t<1>(p, U, x3, st);
    case 2: return launch_spass_h_t<2>(p, U, x3, st);
    case 3: return launch_spass_h_t<3>(p, U, x3, st);
    case 4: return launch_spass_h_t<4>(p, U, x3, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rpca
