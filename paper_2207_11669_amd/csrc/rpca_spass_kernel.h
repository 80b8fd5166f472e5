// S-pass (FP32): the kernel template, shared by the per-tile launches
// (rpca_spass.hip) and the persistent ones (rpca_spass_q.hip).
#pragma once
#include "rpca_device.h"

namespace rpca {



// S-pass epilogue of the FP32 form: the client's U-step term for the
// work-group's 128 rows (Lemma 2's proof for the gradient, argmin_U L_i for
// the closed form). With X = P - c_i U_i (P = Lambda V_i, c_i = rho n_i / n)
// and A_i = (V_i^T V_i + c_i I)^{-1}:
//   GRAD   T = U_i - eta (c_i U_i - P) = U_i + eta X
//   CLOSED T = P A_i + U_i V_i^T V_i A_i = U_i + X A_i
// (V_i^T V_i A_i = I - c_i A_i). ptile holds X (row stride PS), fa A_i in
// FP32 (row stride FS). The closed form runs on FP32 MFMA as (X A_i)^T =
// A_i^T X^T in 16-rank x 16-row tiles: lane l ends with
// (X A_i)[row l%16][rank 16 ct + 4 (l/16) + v] of a tile, and U_i is added
// once at the end (accumulating onto U_i would round every partial sum to
// the size of U_i), so each store covers 16 consecutive rows of a rank
// column. Wave w of phase ph takes the row tiles rt = ph, ph + NPH, ... of
// its 32-row strip.
template <int RT, int NS, int NPH, int PS, int FS>
__device__ __forceinline__ void spass_terms(const DevParams& p, const ClientDev& cl,
                                            const float* __restrict__ U, int b, int w, int phase,
                                            const float* xtile, const float* fa, bool closed) {
  constexpr int RP = 16 * RT;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int MP = p.MP;
  const int row0 = b * kSRows;
  float* __restrict__ Ti = p.P + (int64_t)cl.idx * RP * MP;
  const GLOBAL float* Uc = gptr(U);  // column-major layout, zero past m and r
  const double eta = eta_of_round(p, p.dstate->t);
#pragma unroll
  for (int rt = phase; rt < 2; rt += NPH) {
    const int rl = w * 32 + 16 * rt;  // the tile's first row in the block
    const int64_t grow = row0 + rl + li;
    f4 acc[RT], uv[RT];
#pragma unroll
    for (int ct = 0; ct < RT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) uv[ct][v] = Uc[(int64_t)(16 * ct + 4 * lg + v) * MP + grow];
    const float* xr = xtile + (rl + li) * PS;
    if (closed) {
      // P and U_i are zero past rank r, so the contraction stops at 4 NS.
#pragma unroll
      for (int ct = 0; ct < RT; ++ct) acc[ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int kk = 0; kk < NS; ++kk) {
        const float xb = xr[4 * kk + lg];
#pragma unroll
        for (int ct = 0; ct < RT; ++ct)
          acc[ct] = mfma4(fa[(4 * kk + lg) * FS + 16 * ct + li], xb, acc[ct]);
      }
#pragma unroll
      for (int ct = 0; ct < RT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[ct][v] += uv[ct][v];
    } else {
#pragma unroll
      for (int ct = 0; ct < RT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[ct][v] = (float)((double)uv[ct][v] + eta * (double)xr[16 * ct + 4 * lg + v]);
    }
#pragma unroll
    for (int ct = 0; ct < RT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * ct + 4 * lg + v;
        Ti[(int64_t)c * MP + grow] = c < p.r ? acc[ct][v] : 0.f;
      }
  }
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
// SPLIT: the per-tile form, whose chunk body comes in a copy with and one
// without the Huber sum (see compute_chunk).
// SOUT: what of S the tile writes besides its statistics and U-step term:
// kSOutNone, kSOutDense (column-major into Sout) or kSOutSparse (support
// words and packed nonzero values per 16 x 16 tile, sparse_tile).
// ---------------------------------------------------------------------------
template <int RT, int NS, int SOUT, int NPH, bool SPLIT>
__device__ __forceinline__ void spass_tile(const DevParams& p, const float* __restrict__ Ubase,
                                           int64_t u_stride, float* __restrict__ Sout,
                                           int64_t lds_out, int emit_only, int client_base,
                                           int b, int yi) {
  constexpr int RP = 16 * RT;
  static_assert(NS >= 1 && NS <= 4 * RT, "NS = ceil(r / 4) must fit the rank tiles");
  // P's last rank tile in 4x4 blocks when it holds at most 12 ranks.
  constexpr int NQ = nquads(RP, NS), RTF = NQ ? RT - 1 : RT;
  // Clients run widest first (longest work-groups dispatched earliest), except
  // for the S emission of a client range.
  const ClientDev cl = emit_only ? p.clients[client_base + yi] : p.clients_lpt[yi];
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
  // factor A_i is fetched now (into registers, stored to LDS as FP32 once the
  // ring's first loads are in flight), so the epilogue waits on no memory.
  // Row strides: P (and X) RP + 4 floats, so that a wave's column reads (16
  // rows by 4 ranks) and its accumulator writes (4 rows by 16 ranks) fall in
  // distinct banks; A_i an odd multiple of 16 floats, so that four rows of 16
  // consecutive entries do. 55 KB at r = 64: two work-groups of 256 threads
  // share a compute unit, one's epilogue overlapping the other's sweep.
  constexpr int kPS = RP + 4, kFS = 16 * ((RP / 16) | 1);
  __shared__ float ptile[kSRows * kPS];
  __shared__ float fal[RP * kFS];
  const bool closed = p.u_mode != 0;
  constexpr int kFabPer = (RP * RP + 256 * NPH - 1) / (256 * NPH);
  float fa[kFabPer];
  if (!emit_only && closed) {
    const double* __restrict__ Af = p.Afac + (int64_t)ci * RP * RP;
#pragma unroll
    for (int q = 0; q < kFabPer; ++q) {
      const int e = tid + q * 256 * NPH;
      fa[q] = e < RP * RP ? (float)Af[e] : 0.f;
    }
  }
  auto stage_fa = [&]() {
#pragma unroll
    for (int q = 0; q < kFabPer; ++q) {
      const int e = tid + q * 256 * NPH;
      if (e < RP * RP) fal[(e / RP) * kFS + e % RP] = fa[q];
    }
  };

  double sl2 = 0.0, sl1 = 0.0, shb = 0.0;
  uint32_t nnz = 0;  // wave-uniform count of nonzero S entries
  const bool hub = p.huber != 0;  // Huber sum at the target lambda
  const float lt = p.lam_target;
  const float lam = p.lam;
  constexpr bool STORE = SOUT == kSOutDense;
  GLOBAL float* Sblk = STORE ? gptr_w(Sout) + cl.col0 * lds_out : nullptr;
  // V operands: packed, always in range (lane offset + scalar chunk offset).
  const rsrc_t rVa = make_rsrc(v_fb(p.V, p.NVP, RP) + fb_pa_off(p.NVP, RP), range32((int64_t)p.NVP * 4 * NS * 4));
  const rsrc_t rVb = make_rsrc(v_fb(p.V, p.NVP, RP) + fb_pb_off(p.NVP, RP, NS), range32((int64_t)p.NVP * RP * 4));
  const rsrc_t rVq = make_rsrc(v_fb(p.V, p.NVP, RP) + fb_pq_off(p.NVP, RP, NS), range32((int64_t)p.NVP * 4 * NQ * 4));
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
  // HUB: whether the body sums the Huber function at the target lambda: 0
  // never, 1 always, 2 when the round asks for it (p.huber; the compiler
  // if-converts the test, so the arithmetic runs on every entry). The
  // per-tile form (SPLIT) chooses between bodies 0 and 1 per chunk, a
  // wave-uniform branch, so that rounds at the target lambda skip it; the
  // persistent form keeps body 2, whose loop fits the registers without
  // spilling.
  auto compute_chunk = [&](const Chunk& c, int k, auto hub_tag) {
    constexpr int HUB = decltype(hub_tag)::value;
    const int j0 = (phase + NPH * k) << 4;
    float l2 = 0.f, l1 = 0.f, hb = 0.f;
    // Sparse S of this wave's two 16 x 16 tiles (consecutive tile indices):
    // lane l holds rows l%16 of columns 4 (l/16) + v, so the lanes of quad
    // q = l/4 hold rows 4 (q%4) + e of columns 4 (q/4) + v; a transpose within
    // the quad leaves lane l with slot l (rows 4 (q%4) + e of column
    // 4 (q/4) + l%4). The nonzero slots go to the front of the tile's region
    // in lane order, one float4 store; lane rt keeps tile rt's slot word.
    // Stores go through buffer resources; empty slots take an offset outside
    // the range and write nothing.
    [[maybe_unused]] uint64_t myword = 0;
    // (The row strip via readfirstlane: wave-uniform, so the resources built
    // from it stay in scalar registers.)
    [[maybe_unused]] const int64_t tile0 =
        SOUT == kSOutSparse
            ? sparse_tile(p.MP, cl.vrow0 + j0, __builtin_amdgcn_readfirstlane(arow0))
            : 0;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      f4 a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NS; ++s) a1 = mfma4(c.va[s], ub[rt][s], a1);
      f4 lamv;
      [[maybe_unused]] f4 sv;
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
        if constexpr (HUB == 1) hb += huber1(R, lt);
        if constexpr (HUB == 2) if (hub) hb += huber1(R, lt);
        nnz += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(Sv != 0.f));
        if constexpr (SOUT == kSOutSparse) sv[v] = Sv;
      }
      if constexpr (SOUT == kSOutSparse) {
        const f4 y = quad_transpose(sv);
        const bool ne = y[0] != 0.f || y[1] != 0.f || y[2] != 0.f || y[3] != 0.f;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(ne);
        // This slot goes after every nonzero slot of a lower lane.
        const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        const rsrc_t rSv = make_rsrc(p.Sval + (tile0 + rt) * kSparseVals, kSparseVals * 4u);
        bstore4(rSv, ne ? pos * 16u : kOffNone, y);
        myword = lane == rt ? bal : myword;
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
    shb += (double)hb;
    if constexpr (SOUT == kSOutSparse) {
      // Lanes 0 and 1 write the two tiles' slot words.
      const rsrc_t rSm = make_rsrc(p.Smask + tile0, 2 * 8u);
      bstore64(rSm, lane < 2 ? (uint32_t)lane * 8u : kOffNone, myword);
    }
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
    if (!emit_only && closed) stage_fa();
    __builtin_amdgcn_sched_barrier(0);
    for (int k0 = 0; k0 < nkp; k0 += kSDepth) {
#pragma unroll
      for (int d = 0; d < kSDepth; ++d) {
        const int k = k0 + d;
        if (k < nk) {  // wave-uniform
          if constexpr (!SPLIT)
            compute_chunk(ring[d], k, std::integral_constant<int, 2>{});
          else if (hub)
            compute_chunk(ring[d], k, std::integral_constant<int, 1>{});
          else
            compute_chunk(ring[d], k, std::integral_constant<int, 0>{});
        }
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
    // share of A_i.
    stage_fa();
  }

  if (emit_only) return;
  // Epilogue: P from the two phases' accumulators, summed in LDS in phase
  // order; then X = P - c_i U_i and the client's U-step term for these 128
  // rows. Quads: block b = l/4 summed columns 4 (b/4) + s for rows
  // 4 (b%4) + i; the four column groups (lanes l, l ^ 16, l ^ 32, l ^ 48) are
  // added first.
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
#pragma unroll
  for (int q = 0; q < NPH; ++q) {
    if (phase == q) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
#pragma unroll
        for (int ct = 0; ct < RTF; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float& x = ptile[(w * 32 + 16 * rt + 4 * lg + v) * kPS + 16 * ct + li];
            x = q == 0 ? accp[rt][ct][v] : x + accp[rt][ct][v];
          }
#pragma unroll
        for (int qd = 0; qd < NQ; ++qd)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (lane < 16) {
              float& x = ptile[(w * 32 + 16 * rt + 4 * (lane >> 2) + i) * kPS + 16 * RTF + 4 * qd + (lane & 3)];
              x = q == 0 ? accq[rt][qd][i] : x + accq[rt][qd][i];
            }
      }
    }
    __syncthreads();
  }
  // X = P - c_i U_i, U_i from the MFMA 1 operand registers (rank
  // (l/16) NS + s of row l%16; ranks from 4 NS on are zero in U_i and in P).
  if (phase == 0) {
    const float cf = (float)cl.c;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        float& x = ptile[(w * 32 + 16 * rt + li) * kPS + lg * NS + s];
        x = fmaf(-cf, ub[rt][s], x);
      }
  }
  __syncthreads();
  spass_terms<RT, NS, NPH, kPS, kFS>(p, cl, U, b, w, phase, ptile, fal, closed);
  spass_stats<4 * NPH>(p, ci, b, sl2, sl1, nnz, shb);
}

// The kernel: Q = false, one work-group per tile (grid = row blocks x
// clients); Q = true, a persistent launch whose work-groups take tiles
// t = (row block t % nrb, client t / nrb) from the queue (never for the S
// emission).
template <int RT, int NS, int SOUT, int NPH, bool Q>
__global__ __launch_bounds__(256 * NPH) void k_spass(DevParams p, const float* __restrict__ Ubase,
                                                     int64_t u_stride, float* __restrict__ Sout,
                                                     int64_t lds_out, int emit_only,
                                                     int client_base) {
  if constexpr (!Q) {
    spass_tile<RT, NS, SOUT, NPH, true>(p, Ubase, u_stride, Sout, lds_out, emit_only,
                                         client_base, (int)blockIdx.x, (int)blockIdx.y);
  } else {
    const int ntiles = p.nrb * p.E;
    for (int t = queue_next(p.queue + 2, ntiles); t < ntiles; t = queue_next(p.queue + 2, ntiles))
      spass_tile<RT, NS, SOUT, NPH, false>(p, Ubase, u_stride, Sout, lds_out, 0, 0, t % p.nrb,
                                            t / p.nrb);
  }
}

// S-pass at ranks above kFoldMaxRP, every launch form and output
// (rpca_spass_w.hip).
hipError_t launch_spass_wide(const DevParams& p, const float* U, int64_t u_stride, float* Sout,
                             int64_t lds_out, int emit_only, int client_base, int client_count,
                             hipStream_t st);
// Persistent S-pass launches over all clients from the tile queue
// (rpca_spass_q.hip).
hipError_t launch_spass_queue(const DevParams& p, const float* U, int64_t u_stride,
                              float* Sout, int64_t lds_out, hipStream_t st);
// S-pass over all clients writing sparse S (p.Smask, p.Sval), in the launch
// form p.squeue picks (rpca_spass_s.hip).
hipError_t launch_spass_sparse(const DevParams& p, const float* U, int64_t u_stride,
                               hipStream_t st);

}  // namespace rpca
