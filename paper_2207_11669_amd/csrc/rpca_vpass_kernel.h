// V-pass, streaming part (FP32): the kernel template, shared by the per-tile
// launches (rpca_vpass.hip) and the persistent ones (rpca_vpass_q.hip).
#pragma once
#include "rpca_device.h"

namespace rpca {

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
// MODE kSSparse reads the S the previous S-pass wrote in sparse form (a slot
// word and packed float4 slots per 16 x 16 tile, sparse_tile): lane l's four
// entries are slot b = 16 ((l%16)/4) + 4 (l/16) + (l%16)%4 of the chunk's
// tile, stored (if bit b of the slot word is set) after the tile's nonzero
// slots of lower index: one float4 load.


template <int RT, int NS, int MODE, int KG>
__device__ __forceinline__ void vpass_tile(const DevParams& p, const float* __restrict__ Ubase,
                                           int64_t u_stride, const float* __restrict__ Uold,
                                           const float* __restrict__ Vold, int tile,
                                           float (*red)[16 * RT]) {
  constexpr int RP = 16 * RT;
  static_assert(NS >= 1 && NS <= 4 * RT, "NS = ceil(r / 4) must fit the rank tiles");
  // W's last rank tile in 4x4 blocks when it holds at most 12 ranks.
  constexpr int NQ = nquads(RP, NS), RTF = NQ ? RT - 1 : RT;
  constexpr int kG = KG;                 // column groups per wave
  constexpr int kPh = KG;                // row phases (waves per column set)
  static_assert(KG == 1 || KG == 2 || KG == 4, "column groups per wave");
  const int gx = tile % p.ng64, gy = tile / p.ng64;
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
  const rsrc_t rUb = make_rsrc(gUpb_raw, range32((int64_t)p.MP * RP * 4));
  const rsrc_t rUq = make_rsrc(U + fb_pq_off(p.MP, RP, NS), range32((int64_t)p.MP * 4 * NQ * 4));
  const uint32_t vq_off = (uint32_t)(((lane >> 4) * 4 + (lane & 3)) * 16);
  const rsrc_t rUa = make_rsrc(gUopa_raw, range32((int64_t)p.MP * 4 * NS * 4));
  // Sparse S: the slot words of the next chunk to load are fetched (into
  // scalar registers) one chunk ahead of the values they address.
  constexpr bool SPARSE = MODE == kSSparse;
  const int sp_b = 16 * (li >> 2) + 4 * lg + (li & 3);
  const uint64_t sp_low = ((uint64_t)1 << sp_b) - 1u;
  uint64_t mk[SPARSE ? kG : 1];
  auto load_masks = [&](int k) {
    const int row0 = rbeg + ((ph + kPh * k) << 4);
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int j0 = jw + 16 * g;
      // wave-uniform; column groups past n_i hold no tile of this client
      mk[g] = j0 < cl.n ? *cptr(p.Smask + sparse_tile(p.MP, cl.vrow0 + j0, row0)) : 0;
    }
  };

  // Operands of one 16-row chunk; kVDepth chunks are kept in flight (vector
  // loads complete in order, so everything a chunk needs is issued together).
  struct Chunk {
    f4 m[kG], s[kG];          // M (and stored or sparse S) rows 4*(l/16)..+3 of column 16 g + l%16
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
    if constexpr (SPARSE) {
      // mk holds this chunk's slot words; an empty slot reads 0.
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const int j0 = jw + 16 * g;
        const bool ne = (mk[g] >> sp_b) & 1u;
        const uint32_t pos = (uint32_t)__builtin_popcountll(mk[g] & sp_low);
        const rsrc_t rSv = make_rsrc(p.Sval + sparse_tile(p.MP, cl.vrow0 + j0, row0) * kSparseVals,
                                     kSparseVals * 4u);
        c.s[g] = bload4(rSv, ne ? pos * 16u : kOffNone, 0);
      }
      load_masks(min(k + 1, nk - 1));
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
        for (int e = 0; e < 4; ++e)
          d[e] = c.m[g][e] - ((MODE == kSStored || SPARSE) ? c.s[g][e] : 0.f);
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
    if constexpr (SPARSE) load_masks(0);
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
  // Partial W of the waves, added in LDS (red: kVStreamCols x RP) in
  // row-phase order; the work-group then writes its partial of the 64
  // columns.
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

// The kernel: Q = false, one work-group per tile, tile t = (64-column group
// t % ng64, row split t / ng64); Q = true, a persistent launch whose
// work-groups take tiles in that order from the queue. fin = 1: the first two
// work-groups first run the previous round's finalize (Gram inverse into
// fin_Ginv slot 0; round statistics) while the others stream; nothing in this
// kernel reads what they write, and in a persistent launch they then join the
// queue.
template <int RT, int NS, int MODE, int KG, bool Q>
__global__ __launch_bounds__(256) void k_vpass(DevParams p, const float* __restrict__ Ubase,
                                               int64_t u_stride, const float* __restrict__ Uold,
                                               const float* __restrict__ Vold,
                                               double* __restrict__ fin_Ginv, int fin) {
  // One LDS pool for both roles (sized for this rank, not the largest).
  constexpr int RP = 16 * RT;
  __shared__ double pool[vpass_pool_doubles(RP)];
  float(*red)[RP] = reinterpret_cast<float(*)[RP]>(pool);
  // Ranks above kFoldMaxRP fold no finalize (their launchers pass fin = 0).
  constexpr bool kFold = RP <= kFoldMaxRP;
  if constexpr (!Q) {
    if constexpr (kFold) {
      if (fin && blockIdx.x < 2) {
        finalize_role(p, fin_Ginv, (int)blockIdx.x, pool);
        return;
      }
    }
    vpass_tile<RT, NS, MODE, KG>(p, Ubase, u_stride, Uold, Vold,
                                 (int)blockIdx.x - (kFold && fin ? 2 : 0), red);
  } else {
    if constexpr (kFold)
      if (fin && blockIdx.x < 2) finalize_role(p, fin_Ginv, (int)blockIdx.x, pool);
    const int ntiles = p.ng64 * p.vsplit;
    for (int t = queue_next(p.queue, ntiles); t < ntiles; t = queue_next(p.queue, ntiles))
      vpass_tile<RT, NS, MODE, KG>(p, Ubase, u_stride, Uold, Vold, t, red);
  }
}

// V-pass at ranks above kFoldMaxRP, every launch form (rpca_vpass_w.hip);
// the previous round's finalize has run standalone.
hipError_t launch_vpass_wide(const DevParams& p, int mode, const float* U, int64_t u_stride,
                             const float* Uold, const float* Vold, hipStream_t st);
// Persistent V-pass launches over the tile queue (rpca_vpass_q.hip).
hipError_t launch_vpass_queue(const DevParams& p, int mode, const float* U, int64_t u_stride,
                              const float* Uold, const float* Vold, double* fin_Ginv,
                              hipStream_t st);
// V-pass reading sparse S, in the launch form p.vqueue picks
// (rpca_vpass_s.hip).
hipError_t launch_vpass_sparse(const DevParams& p, const float* U, int64_t u_stride,
                               double* fin_Ginv, hipStream_t st);

}  // namespace rpca
