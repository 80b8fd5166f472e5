// Mixed-precision streaming passes (BF16 and three-product BF16) and the BF16
// copies of M.
#include "rpca_device.h"

namespace rpca {


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
__device__ __forceinline__ void vpass_h_tile(const DevParams& p, const float* __restrict__ Ubase,
                                             const float* __restrict__ Uold,
                                             const float* __restrict__ Vold, int tile,
                                             float (*red)[16 * RT]) {
  constexpr int RP = 16 * RT;
  constexpr int KG = X3 ? 2 : 4, kPh = KG;  // column groups per wave, row phases
  const int gx = tile % p.ng64, gy = tile / p.ng64;
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

  // Operands of one 32-row chunk. M streams from HBM and is kept two chunks
  // ahead (ring of two). The U operands come from L2 and each has a single
  // buffer, refilled for the next chunk right after its last use in this
  // one: the previous U's hP halves (the S rebuild) once the rebuild's MFMA
  // has issued, U's hB once the W products have. Holding them two chunks
  // ahead as well cost 64 registers in three-product rounds (hi and lo) and
  // left one wave per SIMD at r = 64.
  struct MChunk {
    u4 m[KG];                    // BF16 copy: M rows 32 ch + 8 (l/16) + e of column 16 g + l%16
    f4 mf[X3 ? KG : 1][2];       // X3: the same rows in FP32
  };
  struct OpA {
    bf8 uo[2][NK], uol[X3 ? 2 : 1][NK];  // previous U, hP halves (hi, lo)
  };
  struct OpB {
    bf8 u[RT], ul[X3 ? RT : 1];          // U, hB (hi, lo)
  };
  // Three-product rounds up to three rank tiles keep M three chunks ahead
  // (the registers allow it at two waves per SIMD).
  constexpr int kDepth = X3 && RT <= 3 ? 3 : 2;
  MChunk ring[kDepth];
  OpA oa;
  OpB ob;
  auto load_m = [&](MChunk& c, int k) {
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
  };
  auto load_a = [&](OpA& c, int k) {
    if (MODE == kSRecompute) {
      const int ch = ch0 + ph + kPh * k;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
          const int64_t o = (((int64_t)ch * 2 + t) * NK + kb) * 64 + lane;
          c.uo[t][kb] = UohP[o];
          if constexpr (X3) c.uol[t][kb] = UohP[uhl + o];
        }
    }
  };
  auto load_b = [&](OpB& c, int k) {
    const int ch = ch0 + ph + kPh * k;
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) {
      const int64_t o = ((int64_t)ch * RT + ct) * 64 + lane;
      c.u[ct] = UhB[o];
      if constexpr (X3) c.ul[ct] = UhB[uhl + o];
    }
  };
  // The S rebuild's product for every column group: (Uo Vo^T) rows
  // 8 (l/16) + e of column 16 g + l%16, two 16x16 halves.
  f4 o[KG][2];
  auto mfma1 = [&]() {
    if (MODE == kSRecompute) {
#pragma unroll
      for (int g = 0; g < KG; ++g) {
        o[g][0] = f4{0.f, 0.f, 0.f, 0.f};
        o[g][1] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            if constexpr (X3)
              o[g][t] = mfma3(oa.uo[t][kb], oa.uol[t][kb], vb[g][kb], vbl[g][kb], o[g][t]);
            else
              o[g][t] = mfma_bf16(oa.uo[t][kb], vb[g][kb], o[g][t]);
          }
        }
      }
    }
  };
  auto residual_mfma2 = [&](const MChunk& c, int k) {
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
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float a1 = o[g][e >> 2][e & 3];
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
        for (int ct = 0; ct < RT; ++ct) acc[g][ct] = mfma3(dh, dl, ob.u[ct], ob.ul[ct], acc[g][ct]);
      } else {
        const bf8 dh = pack8(d);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) acc[g][ct] = mfma_bf16(dh, ob.u[ct], acc[g][ct]);
      }
    }
  };
  if (nk > 0) {
    // Uniform loop as in k_vpass: every iteration issues the same loads
    // (indices clamped to the wave's last chunk), so the wait counts stay
    // exact; the fences keep each refill where it is written.
    const int nkp = (nk + kDepth - 1) / kDepth * kDepth;
    load_m(ring[0], 0);
    load_a(oa, 0);
    load_b(ob, 0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int d = 1; d < kDepth; ++d) {
      load_m(ring[d], min(d, nk - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int k0 = 0; k0 < nkp; k0 += kDepth) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
        const int k = k0 + d;
        const int kn = min(k + 1, nk - 1);
        if (k < nk) mfma1();  // wave-uniform
        __builtin_amdgcn_sched_barrier(0);
        load_a(oa, kn);
        __builtin_amdgcn_sched_barrier(0);
        if (k < nk) residual_mfma2(ring[d], k);
        __builtin_amdgcn_sched_barrier(0);
        load_b(ob, kn);
        load_m(ring[d], min(k + kDepth, nk - 1));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // Partial W of the waves, added in LDS (red: kVStreamCols x RP) in
  // row-phase order; the work-group then writes its partial of the 64
  // columns.
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

// Work-group roles and tiles as in k_vpass (Q: persistent launch over the
// tile queue).
template <int RT, int NK, int MODE, bool X3, bool Q>
__global__ __launch_bounds__(256) void k_vpass_h(DevParams p, const float* __restrict__ Ubase,
                                                 const float* __restrict__ Uold,
                                                 const float* __restrict__ Vold,
                                                 double* __restrict__ fin_Ginv, int fin) {
  // One LDS pool for both roles (sized for this rank, not the largest).
  constexpr int RP = 16 * RT;
  __shared__ double pool[vpass_pool_doubles(RP)];
  float(*red)[RP] = reinterpret_cast<float(*)[RP]>(pool);
  if constexpr (!Q) {
    if (fin && blockIdx.x < 2) {
      finalize_role(p, fin_Ginv, (int)blockIdx.x, pool);
      return;
    }
    vpass_h_tile<RT, NK, MODE, X3>(p, Ubase, Uold, Vold, (int)blockIdx.x - (fin ? 2 : 0), red);
  } else {
    if (fin && blockIdx.x < 2) finalize_role(p, fin_Ginv, (int)blockIdx.x, pool);
    const int ntiles = p.ng64 * p.vsplit;
    for (int t = queue_next(p.queue, ntiles); t < ntiles; t = queue_next(p.queue, ntiles))
      vpass_h_tile<RT, NK, MODE, X3>(p, Ubase, Uold, Vold, t, red);
  }
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
// holds P and an FP32 copy of A_i (54 KB at r = 64), so two
// work-groups fit on a compute unit and one's epilogue overlaps the other's
// sweep.
// ---------------------------------------------------------------------------
// HUB: 0, the Huber sum at the target lambda is left out (rounds at the
// target lambda); 1, it is taken; 2, p.huber decides per round (the test is
// if-converted, so its arithmetic runs on every entry).
template <int RT, int NK, bool X3, int HUB>
__device__ __forceinline__ void spass_h_tile(const DevParams& p, const float* __restrict__ U, int b,
                                             int yi) {
  constexpr int RP = 16 * RT;
  constexpr int kRT = X3 ? 2 : 4;   // 16-row tiles per wave
  constexpr int kPh = X3 ? 1 : 2;   // column phases
  constexpr int kRG = 4 / kPh;      // row groups of 16 kRT rows
  static_assert(kRG * 16 * kRT == kSRows, "row groups cover the work-group's rows");
  const ClientDev cl = p.clients_lpt[yi];
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
    // Negated once: MFMA 1 then accumulates M - U V^T onto M (the residual
    // needs no subtraction per entry; the pass is VALU-bound).
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        ub[rt][kb] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4, ub[rt][kb]) ^ 0x80008000u);
        if constexpr (X3)
          ubl[rt][kb] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4, ubl[rt][kb]) ^ 0x80008000u);
      }
  }
  f4 accp[kRT][RT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) accp[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};

  // A_i of the closed-form step, rounded to FP32, for the epilogue (made
  // visible by the barriers that add the phases' P). Rows are padded to an
  // odd multiple of 16 floats, so that the epilogue's operand reads (four
  // rows of 16 consecutive entries per wave) fall in distinct banks.
  constexpr int kFS = 16 * ((RP / 16) | 1);
  __shared__ float fal[RP * kFS];
  const bool closed = p.u_mode != 0;
  if (closed) {
    const double* __restrict__ Af = p.Afac + (int64_t)ci * RP * RP;
    for (int e = tid; e < RP * RP; e += blockDim.x) fal[(e / RP) * kFS + e % RP] = (float)Af[e];
  }

  double sl2 = 0.0, sl1 = 0.0, shb = 0.0;
  uint32_t nnz = 0;
  const float lam = p.lam;
  const bool hub = p.huber != 0;  // Huber sum at the target lambda
  const float lt = p.lam_target;
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
  // Operands of one 32-column chunk. M streams from HBM and is kept two
  // chunks ahead (ring of two). The V operands come from L2. In one-product
  // rounds they ride in the same ring. In three-product rounds each has a
  // single buffer, refilled for the next chunk right after its last use in
  // this one: the hP halves (MFMA 1) once MFMA 1 has issued, hB (MFMA 2) once
  // MFMA 2 has. Holding them two chunks ahead there cost 64 registers (hi and
  // lo) and left one wave per SIMD at r = 64; with one-product rounds the
  // single buffers left the L2 latency of every chunk exposed (S-pass 1.12 ->
  // 1.82 ms at 20000 x 100000, r = 64).
  struct MChunk {
    u4 m[kRT];                  // M[row arow0 + 16 rt + l%16][col 32 cc + 8 (l/16) + e]
    float mf[X3 ? kRT : 1][8];  // X3: the same entries in FP32
  };
  struct OpA {
    bf8 va[2][NK], val[X3 ? 2 : 1][NK];  // V hP halves (hi, lo)
  };
  struct OpB {
    bf8 vb[RT], vbl[X3 ? RT : 1];        // V hB (hi, lo)
  };
  constexpr int kDepth = 2;
  constexpr int kOD = X3 ? 1 : 2;  // V operand buffers
  MChunk ring[kDepth];
  OpA oa[kOD];
  OpB ob[kOD];
  const int nch = (cl.n + 31) >> 5;
  const int nk = (nch - phase + kPh - 1) / kPh;  // chunks phase, phase + kPh, ... below nch
  auto load_m = [&](MChunk& c, int k) {
    const int cc = phase + kPh * k;
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
  };
  auto load_a = [&](OpA& c, int k) {
    const int64_t vch = (cl.vrow0 >> 5) + phase + kPh * k;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        const int64_t o = ((vch * 2 + t) * NK + kb) * 64 + lane;
        c.va[t][kb] = VhP[o];
        if constexpr (X3) c.val[t][kb] = VhP[vhl + o];
      }
  };
  auto load_b = [&](OpB& c, int k) {
    const int64_t vch = (cl.vrow0 >> 5) + phase + kPh * k;
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) {
      const int64_t o = (vch * RT + ct) * 64 + lane;
      c.vb[ct] = VhB[o];
      if constexpr (X3) c.vbl[ct] = VhB[vhl + o];
    }
  };
  // MFMA 1 for every row tile: the residual's transpose M^T - (U V^T)^T in
  // two 16x16 halves per tile, the accumulators starting from the lane's
  // entries of M (rows 8 (l/16) + e of the chunk's columns) and the U
  // operand negated.
  f4 o[kRT][2];
  auto init_o = [&](const MChunk& c, int rt) {
    float x[8];
    if constexpr (X3) {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = c.mf[rt][e];
    } else {
      unpack8(c.m[rt], x);
    }
    o[rt][0] = f4{x[0], x[1], x[2], x[3]};
    o[rt][1] = f4{x[4], x[5], x[6], x[7]};
  };
  auto mfma1 = [&](const MChunk& c, const OpA& a) {
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      init_o(c, rt);
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if constexpr (X3)
            o[rt][t] = mfma3(a.va[t][kb], a.val[t][kb], ub[rt][kb], ubl[rt][kb], o[rt][t]);
          else
            o[rt][t] = mfma_bf16(a.va[t][kb], ub[rt][kb], o[rt][t]);
        }
      }
    }
  };
  // Residual, soft-threshold and statistics per row tile, then MFMA 2; with
  // FUSED, each row tile's MFMA 1 runs just before its threshold, so only one
  // tile's (U V^T)^T is live at a time.
  auto threshold_mfma2 = [&](const MChunk& c, const OpA& oa, const OpB& ob, auto fused) {
    constexpr bool FUSED = decltype(fused)::value;
    float l2 = 0.f, l1 = 0.f, hb = 0.f;
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      if constexpr (FUSED) {
        init_o(c, rt);
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            if constexpr (X3)
              o[rt][t] = mfma3(oa.va[t][kb], oa.val[t][kb], ub[rt][kb], ubl[rt][kb], o[rt][t]);
            else
              o[rt][t] = mfma_bf16(oa.va[t][kb], ub[rt][kb], o[rt][t]);
          }
        }
      }
      float lamv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float R = o[rt][e >> 2][e & 3];
        const float L = __builtin_amdgcn_fmed3f(R, -lam, lam);  // clip(R, -lam, lam)
        const float Sv = R - L;
        lamv[e] = L;
        l2 = fmaf(L, L, l2);
        l1 += fabsf(Sv);
        if constexpr (HUB == 1) hb += huber1(R, lt);
        if constexpr (HUB == 2) if (hub) hb += huber1(R, lt);
        nnz += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(Sv != 0.f));
      }
      if constexpr (X3) {
        bf8 lh, ll;
        split8(lamv, lh, ll);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) accp[rt][ct] = mfma3(lh, ll, ob.vb[ct], ob.vbl[ct], accp[rt][ct]);
      } else {
        const bf8 lh = pack8(lamv);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) accp[rt][ct] = mfma_bf16(lh, ob.vb[ct], accp[rt][ct]);
      }
    }
    sl2 += (double)l2;
    sl1 += (double)l1;
    shb += (double)hb;
  };
  if (nk > 0) {
    // Uniform loop: every iteration issues the same loads (chunk indices
    // clamped to the wave's last chunk), so the wait counts stay exact, and
    // the fences keep each refill where it is written (left alone, the
    // scheduler sinks loads towards their first use).
    const int nkp = (nk + kDepth - 1) / kDepth * kDepth;
    if constexpr (kOD == 1) {
      load_m(ring[0], 0);
      load_a(oa[0], 0);
      load_b(ob[0], 0);
      __builtin_amdgcn_sched_barrier(0);
      load_m(ring[1], min(1, nk - 1));
      __builtin_amdgcn_sched_barrier(0);
      for (int k0 = 0; k0 < nkp; k0 += kDepth) {
#pragma unroll
        for (int d = 0; d < kDepth; ++d) {
          const int k = k0 + d;
          const int kn = min(k + 1, nk - 1);
          if (k < nk) mfma1(ring[d], oa[0]);  // wave-uniform
          __builtin_amdgcn_sched_barrier(0);
          load_a(oa[0], kn);
          __builtin_amdgcn_sched_barrier(0);
          if (k < nk) threshold_mfma2(ring[d], oa[0], ob[0], std::false_type{});
          __builtin_amdgcn_sched_barrier(0);
          load_b(ob[0], kn);
          load_m(ring[d], min(k + kDepth, nk - 1));
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
      // Every operand of a chunk in the same ring slot, issued together.
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
        const int k = min(d, nk - 1);
        load_m(ring[d], k);
        load_a(oa[d], k);
        load_b(ob[d], k);
        __builtin_amdgcn_sched_barrier(0);
      }
      for (int k0 = 0; k0 < nkp; k0 += kDepth) {
#pragma unroll
        for (int d = 0; d < kDepth; ++d) {
          const int k = k0 + d;
          if (k < nk) threshold_mfma2(ring[d], oa[d], ob[d], std::true_type{});  // wave-uniform
          __builtin_amdgcn_sched_barrier(0);
          const int kn = min(k + kDepth, nk - 1);
          load_m(ring[d], kn);
          load_a(oa[d], kn);
          load_b(ob[d], kn);
          __builtin_amdgcn_sched_barrier(0);
        }
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
    // T_i = P A_i + U_i V_i^T V_i A_i = U_i + X A_i with X = P - c_i U_i
    // (V_i^T V_i A_i = I - c_i A_i), on FP32 MFMA as (X A_i)^T = A_i^T X^T in
    // 16-rank x 16-row tiles, U_i added at the end: wave wv takes rows
    // 32 wv .. +31 of the block, and lane l ends with
    // T[row l%16][rank 4 (l/16) + v] of a tile, so each store covers 16
    // consecutive rows of a rank column. P comes from LDS, U_i (FP32) from its
    // column-major layout; both are zero past rank r, so the contraction stops
    // at 4 ceil(r/4).
    const int kK = (p.r + 3) / 4;
    const int rb = 32 * wv;
    const GLOBAL float* Uc = gptr(U) + row0 + rb + li;
    const float cf = (float)cl.c;
    f4 acc[2][RT];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < RT; ++ct) acc[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int kk = 0; kk < kK; ++kk) {
      float xb[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
        xb[rt] = fmaf(-cf, Uc[(int64_t)(4 * kk + lg) * MP + 16 * rt],
                      ptile[rb + 16 * rt + li][4 * kk + lg]);
#pragma unroll
      for (int ct = 0; ct < RT; ++ct) {
        const float a0 = fal[(4 * kk + lg) * kFS + 16 * ct + li];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) acc[rt][ct] = mfma4(a0, xb[rt], acc[rt][ct]);
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < RT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * ct + 4 * lg + v;
          const float t = acc[rt][ct][v] + Uc[(int64_t)c * MP + 16 * rt];
          Ti[(int64_t)c * MP + row0 + rb + 16 * rt + li] = c < p.r ? t : 0.f;
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
  spass_stats<4>(p, ci, b, sl2, sl1, nnz, shb);
}

// One work-group per tile (grid = row blocks x clients), or (Q) a persistent
// launch over the tile queue, tiles as in k_spass.
// The per-tile form asks for two work-groups per compute unit (the LDS
// allows it): at most 256 registers per lane, which it fits without spilling,
// so that one work-group's epilogue overlaps the other's sweep. The queue
// form's loop needs more registers and keeps the default bound.
// The per-tile form comes in two instantiations, with and without the Huber
// sum, picked at launch; the queue form decides per round.
template <int RT, int NK, bool X3, int HUB>
__global__ __launch_bounds__(256, 2) void k_spass_h_tile(DevParams p, const float* __restrict__ U) {
  spass_h_tile<RT, NK, X3, HUB>(p, U, (int)blockIdx.x, (int)blockIdx.y);
}
template <int RT, int NK, bool X3>
__global__ __launch_bounds__(256) void k_spass_h_queue(DevParams p, const float* __restrict__ U) {
  const int ntiles = p.nrb * p.E;
  for (int t = queue_next(p.queue + 2, ntiles); t < ntiles; t = queue_next(p.queue + 2, ntiles))
    spass_h_tile<RT, NK, X3, 2>(p, U, t % p.nrb, t / p.nrb);
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
  const int ntiles = p.ng64 * p.vsplit;
  // The first round (S = 0) always runs one work-group per tile.
  auto go = [&](auto m, auto x) {
    constexpr int kMode = decltype(m)::value;
    constexpr bool kX3 = decltype(x)::value;
    if (kMode == kSRecompute && p.vqueue) {
      auto kernel = k_vpass_h<RT, NK, kSRecompute, kX3, true>;
      const int groups = pass_groups(kernel, 256, ntiles, 1);
      hipLaunchKernelGGL(kernel, dim3((unsigned)(groups + 2 * fin)), dim3(256), 0, st, p, U, Uold,
                         Vold, fin_Ginv, fin);
    } else {
      hipLaunchKernelGGL((k_vpass_h<RT, NK, kMode, kX3, false>), dim3((unsigned)(ntiles + 2 * fin)),
                         dim3(256), 0, st, p, U, Uold, Vold, fin_Ginv, fin);
    }
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
  const int ntiles = p.nrb * p.E;
  auto go = [&](auto persistent, auto per_tile, auto per_tile_huber) {
    if (p.squeue) {
      const int groups = pass_groups(persistent, 256, ntiles, 1);
      hipLaunchKernelGGL(persistent, dim3(groups), dim3(256), 0, st, p, U);
    } else {
      hipLaunchKernelGGL(p.huber ? per_tile_huber : per_tile, dim3(p.nrb, p.E), dim3(256), 0, st,
                         p, U);
    }
  };
  if (x3)
    go(k_spass_h_queue<RT, NK, true>, k_spass_h_tile<RT, NK, true, 0>,
       k_spass_h_tile<RT, NK, true, 1>);
  else
    go(k_spass_h_queue<RT, NK, false>, k_spass_h_tile<RT, NK, false, 0>,
       k_spass_h_tile<RT, NK, false, 1>);
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
