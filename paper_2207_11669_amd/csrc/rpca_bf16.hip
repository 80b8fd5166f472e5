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
// itself, so a wave takes all four 16-column groups of the tile, which share
// the chunk's U operands in registers, and the four waves split the rows
// (phase q takes chunks q, q + 4, ...); their partial W are added in LDS in
// phase order at the end. M comes from the V-pass BF16 copy (one 16-byte
// load per lane), and every contraction is one BF16 product.
// Lane l holds rows 8 (l/16) + e of column 16 g + l%16: the A operand of W's
// MFMA, with U's hB packing as B; accumulator W[col 16 g + 4 (l/16) + v]
// [rank 16 ct + l%16]. kSRecompute rebuilds S = soft(M - Uo Vo^T): two 16x16
// products per chunk and column group with the previous U's hP packing on the
// A side and the previous V's hA packing on the B side leave lane l the same
// eight rows of its column.
// ---------------------------------------------------------------------------
template <int RT, int NK, int MODE>
__device__ __forceinline__ void vpass_h_tile(const DevParams& p, const float* __restrict__ Ubase,
                                             const float* __restrict__ Uold,
                                             const float* __restrict__ Vold, int tile,
                                             float (*red)[16 * RT]) {
  constexpr int RP = 16 * RT;
  constexpr int KG = 4, kPh = 4;  // column groups per wave, row phases
  const int gx = tile % p.ng64, gy = tile / p.ng64;
  const VTile vt = p.vg64[gx];
  const ClientDev& cl = vt.cl;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int ph = __builtin_amdgcn_readfirstlane(tid >> 6);  // row phase
  const int jw = vt.j0;                                     // first column of every wave
  const float lam = p.lam;
  const int MP = p.MP;

  const GLOBAL bf8* UhB = reinterpret_cast<const GLOBAL bf8*>(gptr(u_hb(Ubase, p))) +
                          2 * (int64_t)MP * p.RK / 8;
  const GLOBAL bf8* UohP = reinterpret_cast<const GLOBAL bf8*>(gptr(u_hb(Uold, p))) +
                           (int64_t)MP * p.RK / 8;
  bf8 vb[KG][NK];  // S rebuild B operand: Vo[col][rank 32 kb + 8 (l/16) + e]
  if (MODE == kSRecompute) {
    const GLOBAL bf8* VohA = reinterpret_cast<const GLOBAL bf8*>(gptr(v_hb(Vold, p)));
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const int vch = (cl.vrow0 + jw + 16 * g) >> 4;
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) vb[g][kb] = VohA[((int64_t)vch * NK + kb) * 64 + lane];
    }
  }
  const int rbeg = gy * p.vsplit_rows;
  const int rend = min(p.m, rbeg + p.vsplit_rows);
  const int ch0 = rbeg >> 5;
  const int nch = (rend - rbeg + 31) >> 5;
  const int nk = (nch - ph + kPh - 1) / kPh;  // this wave's chunks ph, ph + kPh, ...
  // M: the BF16 copy, column group cg = (jw + 16 g) / 16.
  const GLOBAL u4* Mv = reinterpret_cast<const GLOBAL u4*>(gptr(p.Mbv)) +
                        (int64_t)cl.vrow0 * MP / 8 + (int64_t)(jw >> 4) * (MP >> 5) * 64 + lane;
  const int64_t gstride = (int64_t)(MP >> 5) * 64;  // u4 units between column groups
  f4 acc[KG][RT];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) acc[g][ct] = f4{0.f, 0.f, 0.f, 0.f};

  // Operands of one 32-row chunk. M streams from HBM and is kept two chunks
  // ahead (ring of two). The U operands come from L2 and each has a single
  // buffer, refilled for the next chunk right after its last use in this
  // one: the previous U's hP halves (the S rebuild) once the rebuild's MFMA
  // has issued, U's hB once the W products have.
  struct MChunk {
    u4 m[KG];  // M rows 32 ch + 8 (l/16) + e of column 16 g + l%16
  };
  struct OpA {
    bf8 uo[2][NK];  // previous U, hP halves
  };
  struct OpB {
    bf8 u[RT];  // U, hB
  };
  constexpr int kDepth = 2;
  MChunk ring[kDepth];
  OpA oa;
  OpB ob;
  auto load_m = [&](MChunk& c, int k) {
    const int ch = ch0 + ph + kPh * k;
#pragma unroll
    for (int g = 0; g < KG; ++g) c.m[g] = Mv[g * gstride + (int64_t)ch * 64];
  };
  auto load_a = [&](OpA& c, int k) {
    if (MODE == kSRecompute) {
      const int ch = ch0 + ph + kPh * k;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) c.uo[t][kb] = UohP[(((int64_t)ch * 2 + t) * NK + kb) * 64 + lane];
    }
  };
  auto load_b = [&](OpB& c, int k) {
    const int ch = ch0 + ph + kPh * k;
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) c.u[ct] = UhB[((int64_t)ch * RT + ct) * 64 + lane];
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
        for (int kb = 0; kb < NK; ++kb)
#pragma unroll
          for (int t = 0; t < 2; ++t) o[g][t] = mfma_bf16(oa.uo[t][kb], vb[g][kb], o[g][t]);
      }
    }
  };
  auto residual_mfma2 = [&](const MChunk& c) {
    // Rows past m and columns past n_i are zero in the BF16 copy and in the
    // factors' packings, so they give d = 0 without a mask.
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      float x[8], d[8];
      unpack8(c.m[g], x);
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
      const bf8 dh = pack8(d);
#pragma unroll
      for (int ct = 0; ct < RT; ++ct) acc[g][ct] = mfma_bf16(dh, ob.u[ct], acc[g][ct]);
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
    load_m(ring[1], min(1, nk - 1));
    __builtin_amdgcn_sched_barrier(0);
    for (int k0 = 0; k0 < nkp; k0 += kDepth) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
        const int k = k0 + d;
        const int kn = min(k + 1, nk - 1);
        if (k < nk) mfma1();  // wave-uniform
        __builtin_amdgcn_sched_barrier(0);
        load_a(oa, kn);
        __builtin_amdgcn_sched_barrier(0);
        if (k < nk) residual_mfma2(ring[d]);
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
  for (int q0 = 0; q0 < kPh; ++q0) {
    if (ph == q0) {
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int ct = 0; ct < RT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float& x = red[16 * g + 4 * lg + v][16 * ct + li];
            x = q0 == 0 ? acc[g][ct][v] : x + acc[g][ct][v];
          }
    }
    __syncthreads();
  }
  GLOBAL float* wp = gptr_w(p.Wpart) + ((int64_t)gy * p.NVP + cl.vrow0 + vt.j0) * RP;
  for (int e = tid; e < kVStreamCols * RP; e += blockDim.x) wp[e] = red[e / RP][e % RP];
}

// ---------------------------------------------------------------------------
// BF16 V-pass with the U operands staged in LDS (three-product rounds
// always; one-product rounds with one column group). Loads of one wave
// complete in issue order, so in the register form every wait for a U
// operand (an L2 hit, fetched one chunk ahead) also waits for the M chunks
// issued before it, and M effectively streams one chunk ahead whatever the
// ring depth. Here a work-group takes KT 64-column tiles over the same
// rows, each of its four waves one 16-column group of every tile, so a
// chunk's U operands (previous U hP, U hB, hi and in three-product rounds lo:
// 8-16 KiB) are needed once per work-group: the waves copy them from L2
// straight into LDS (global_load_lds, 1 KiB per instruction, no registers),
// kLdsStages chunks ahead, and issue each chunk's M loads beside its copies.
// A chunk's group of loads is waited for as a whole, kLdsStages - 2 groups
// behind the newest, so both M and U stream kLdsStages - 1 chunks ahead. One
// barrier per chunk makes the other waves' copies visible and frees the
// stage read in the chunk before. Per wave and chunk: one or two 16-byte
// loads of M per tile, a quarter of the copies, and one 16-byte LDS read per
// U operand.
// ---------------------------------------------------------------------------
constexpr int kLdsStages = 4;
// 1 KiB units of a chunk's U operands: the previous U's hP halves (S rebuild
// only; hi, then lo in three-product rounds), then U's hB (hi, then lo); and
// the bytes of one stage, the units rounded up to a multiple of the four
// waves.
template <int RT, int NK, int MODE, bool X3>
constexpr int vpass_h3_units() {
  return ((MODE == kSRecompute ? 2 * NK : 0) + RT) * (X3 ? 2 : 1);
}
template <int RT, int NK, int MODE, bool X3>
constexpr int vpass_h3_stage_bytes() {
  return (vpass_h3_units<RT, NK, MODE, X3>() + 3) / 4 * 4 * 1024;
}

typedef __attribute__((address_space(3))) void lds_void;
__device__ __forceinline__ uint32_t lds_addr(void* p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char*)p;
}
// N 16-byte LDS reads at a + 1024 i, completed before the block ends: the
// compiler, which does not see the reads, then cannot place a wait for the
// LDS copies of later chunks in front of them.
template <int N>
__device__ __forceinline__ void lds_read_1k(u4* o, uint32_t a);
template <>
__device__ __forceinline__ void lds_read_1k<1>(u4* o, uint32_t a) {
  asm volatile(
      "ds_read_b128 %0, %1\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0])
      : "v"(a)
      : "memory");
}
template <>
__device__ __forceinline__ void lds_read_1k<3>(u4* o, uint32_t a) {
  asm volatile(
      "ds_read_b128 %0, %3\n\t"
      "ds_read_b128 %1, %3 offset:1024\n\t"
      "ds_read_b128 %2, %3 offset:2048\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2])
      : "v"(a)
      : "memory");
}
template <>
__device__ __forceinline__ void lds_read_1k<2>(u4* o, uint32_t a) {
  asm volatile(
      "ds_read_b128 %0, %2\n\t"
      "ds_read_b128 %1, %2 offset:1024\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0]), "=&v"(o[1])
      : "v"(a)
      : "memory");
}
template <>
__device__ __forceinline__ void lds_read_1k<4>(u4* o, uint32_t a) {
  asm volatile(
      "ds_read_b128 %0, %4\n\t"
      "ds_read_b128 %1, %4 offset:1024\n\t"
      "ds_read_b128 %2, %4 offset:2048\n\t"
      "ds_read_b128 %3, %4 offset:3072\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3])
      : "v"(a)
      : "memory");
}
template <>
__device__ __forceinline__ void lds_read_1k<6>(u4* o, uint32_t a) {
  asm volatile(
      "ds_read_b128 %0, %6\n\t"
      "ds_read_b128 %1, %6 offset:1024\n\t"
      "ds_read_b128 %2, %6 offset:2048\n\t"
      "ds_read_b128 %3, %6 offset:3072\n\t"
      "ds_read_b128 %4, %6 offset:4096\n\t"
      "ds_read_b128 %5, %6 offset:5120\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5])
      : "v"(a)
      : "memory");
}
template <>
__device__ __forceinline__ void lds_read_1k<8>(u4* o, uint32_t a) {
  asm volatile(
      "ds_read_b128 %0, %8\n\t"
      "ds_read_b128 %1, %8 offset:1024\n\t"
      "ds_read_b128 %2, %8 offset:2048\n\t"
      "ds_read_b128 %3, %8 offset:3072\n\t"
      "ds_read_b128 %4, %8 offset:4096\n\t"
      "ds_read_b128 %5, %8 offset:5120\n\t"
      "ds_read_b128 %6, %8 offset:6144\n\t"
      "ds_read_b128 %7, %8 offset:7168\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]),
        "=&v"(o[6]), "=&v"(o[7])
      : "v"(a)
      : "memory");
}
// s_waitcnt immediate that waits until at most n vector-memory operations of
// the wave are outstanding (n < 64) and leaves the other counters alone. The
// builtin form lets the compiler account for the wait in its own ones.
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
// Barrier of the work-group's waves without a memory fence (a fence would
// wait for every load in flight); as a compiler barrier it keeps memory
// operations on their side of it.
__device__ __forceinline__ void bare_barrier() { asm volatile("s_barrier" ::: "memory"); }
// A buffer resource whose operands are made wave-uniform, so that it lives
// in scalar registers (the compiler cannot tell that values read from the
// tile table are the same in every lane, and would otherwise loop over the
// lanes at each load).
__device__ __forceinline__ rsrc_t uniform_rsrc(const void* base, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return make_rsrc(reinterpret_cast<const void*>(((uint64_t)hi << 32) | lo),
                   __builtin_amdgcn_readfirstlane(bytes));
}

// Tiles per work-group of the staged V-pass: KT consecutive 64-column tiles
// over the same rows (clients may differ; the U operands are the same), so
// that each wave streams KT column groups of M against one copy of a chunk's
// U operands. The launch picks KT from the column-group knob: one-product
// rounds 4; three-product rounds (FP32 M, hi and lo operands) 2, or 1 with
// one column group.
__host__ __device__ inline int vpass_h3_groups(int ng64, int kt) { return (ng64 + kt - 1) / kt; }

template <int RT, int NK, int MODE, bool X3, int KT>
__device__ __forceinline__ void vpass_h3_tile(const DevParams& p, const float* __restrict__ Ubase,
                                              const float* __restrict__ Uold,
                                              const float* __restrict__ Vold, int tile,
                                              float (*red)[16 * RT], void* stage_mem) {
  constexpr int RP = 16 * RT;
  constexpr int kX = X3 ? 2 : 1;          // hi, and lo in three-product rounds
  constexpr bool kA = MODE == kSRecompute;
  constexpr int kUA = kA ? 2 * NK * kX : 0;  // 1 KiB units of the previous U (hP)
  constexpr int kUnits = vpass_h3_units<RT, NK, MODE, X3>();  // and of U (hB)
  constexpr int kPerWave = (kUnits + 3) / 4;
  constexpr int kStage = vpass_h3_stage_bytes<RT, NK, MODE, X3>();
  static_assert(kStage == 4 * kPerWave * 1024, "one padded unit per wave and copy");
  constexpr int kD = kLdsStages - 1;     // chunks ahead (M ring depth)
  const int ngr = vpass_h3_groups(p.ng64, KT);
  const int gx0 = (tile % ngr) * KT, gy = tile / ngr;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const float lam = p.lam;
  const int MP = p.MP;
  // Tile t of the group (past the last tile: the last again, reading 0 and
  // writing nothing); wave w takes its column group w.
  bool valid[KT];
  int jw[KT];
  const ClientDev* clp[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    valid[t] = gx0 + t < p.ng64;
    const VTile& vt = p.vg64[min(gx0 + t, p.ng64 - 1)];
    clp[t] = &vt.cl;
    jw[t] = vt.j0 + 16 * w;
  }

  const int64_t uhl = hb_elems(MP, p.RK, p.RP) / 8, vhl = hb_elems(p.NVP, p.RK, p.RP) / 8;
  const GLOBAL bf8* UhB = reinterpret_cast<const GLOBAL bf8*>(gptr(u_hb(Ubase, p))) +
                          2 * (int64_t)MP * p.RK / 8;
  const GLOBAL bf8* UohP = reinterpret_cast<const GLOBAL bf8*>(gptr(u_hb(Uold, p))) +
                           (int64_t)MP * p.RK / 8;
  // S rebuild B operand (hi, lo): Vo[col][rank 32 kb + 8 (l/16) + e]
  bf8 vb[KT][NK], vbl[X3 ? KT : 1][NK];
  if (kA) {
    const GLOBAL bf8* VohA = reinterpret_cast<const GLOBAL bf8*>(gptr(v_hb(Vold, p)));
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const int vch = (clp[t]->vrow0 + jw[t]) >> 4;
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        vb[t][kb] = VohA[((int64_t)vch * NK + kb) * 64 + lane];
        if constexpr (X3) vbl[t][kb] = VohA[vhl + ((int64_t)vch * NK + kb) * 64 + lane];
      }
    }
  }
  const int rbeg = gy * p.vsplit_rows;
  const int rend = min(p.m, rbeg + p.vsplit_rows);
  const int ch0 = rbeg >> 5;
  const int nk = (rend - rbeg + 31) >> 5;  // chunks of the row split (the same for every wave)
  // M: (X3) the caller's FP32 block through one buffer resource per tile
  // (columns past n_i, and every column of a tile past the last, read 0;
  // rows past m are masked in the last chunk), or the V-pass BF16 copy, one
  // 16-byte load per lane (zero past m and n_i; a tile past the last reads
  // the last tile's and its W is not written).
  rsrc_t rM[X3 ? KT : 1];
  uint32_t vM[X3 ? KT : 1];
  const GLOBAL u4* Mv[X3 ? 1 : KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const ClientDev& cl = *clp[t];
    if constexpr (X3) {
      rM[t] = uniform_rsrc(cl.M + (int64_t)min(jw[t], cl.n) * cl.ldm,
                           valid[t] ? block_bytes_from(cl.n, jw[t], cl.ldm) : 0u);
      vM[t] = (uint32_t)(li * cl.ldm) * 4u;
    } else {
      Mv[t] = reinterpret_cast<const GLOBAL u4*>(gptr(p.Mbv)) + (int64_t)cl.vrow0 * MP / 8 +
              (int64_t)(jw[t] >> 4) * (MP >> 5) * 64 + lane;
    }
  }

  // The units this wave copies (u = w, w + 4, ...): source of chunk 0 and
  // the stride between chunks, in 16-byte elements. Unit u of a stage is
  // the wave operand read at stage + 1024 u + 16 lane. Every wave issues
  // kPerWave copies, so that the count of loads per chunk is a constant;
  // units past the last (when 4 does not divide their count) copy the last
  // unit again into padding slots that nothing reads.
  const GLOBAL bf8* src[kPerWave];
  int cstr[kPerWave];
#pragma unroll
  for (int i = 0; i < kPerWave; ++i) {
    const int u = min(w + 4 * i, kUnits - 1);
    if (kA && u < 2 * NK) {
      src[i] = UohP + u * 64 + lane;
      cstr[i] = 2 * NK * 64;
    } else if (kA && u < kUA) {
      src[i] = UohP + uhl + (u - 2 * NK) * 64 + lane;
      cstr[i] = 2 * NK * 64;
    } else if (u < kUA + RT) {
      src[i] = UhB + (u - kUA) * 64 + lane;
      cstr[i] = RT * 64;
    } else {
      src[i] = UhB + uhl + (u - kUA - RT) * 64 + lane;
      cstr[i] = RT * 64;
    }
  }
  char* const stages = reinterpret_cast<char*>(stage_mem);
  const uint32_t stage_lds = lds_addr(stage_mem) + 16u * (uint32_t)lane;
  // Copies of chunk k's U operands (the last chunk past the end) into stage
  // k mod kLdsStages.
  auto copy_u = [&](int k) {
    const int ch = ch0 + min(k, nk - 1);
    char* st = stages + (k % kLdsStages) * kStage;
#pragma unroll
    for (int i = 0; i < kPerWave; ++i)
      __builtin_amdgcn_global_load_lds((GLOBAL void*)(src[i] + (int64_t)ch * cstr[i]),
                                       (lds_void*)(st + (w + 4 * i) * 1024), 16, 0, 0);
  };
  // M rows 32 ch + 8 (l/16) + e of column jw[t] + l%16: FP32 (X3, two
  // 16-byte loads) or BF16 (one).
  u4 ring[kD][KT][kX];
  auto load_m = [&](u4 (*c)[kX], int k) {
    const int ch = ch0 + min(k, nk - 1);
    if constexpr (X3) {
      const uint32_t rowb = (uint32_t)(32 * ch + 8 * lg) * 4u;
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        c[t][0] = __builtin_bit_cast(u4, bload4(rM[t], vM[t] + rowb, 0));
        c[t][kX - 1] = __builtin_bit_cast(u4, bload4(rM[t], vM[t] + rowb + 16u, 0));
      }
    } else {
#pragma unroll
      for (int t = 0; t < KT; ++t) c[t][0] = Mv[t][(int64_t)ch * 64];
    }
  };
  f4 acc[KT][RT];
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) acc[t][ct] = f4{0.f, 0.f, 0.f, 0.f};

  auto chunk = [&](const u4 (*c)[kX], int k) {
    const uint32_t sa = stage_lds + (uint32_t)((k % kLdsStages) * kStage);
    f4 o[KT][2];
#pragma unroll
    for (int t = 0; t < KT; ++t) o[t][0] = o[t][1] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (kA) {
      // (Uo Vo^T) rows 8 (l/16) + e of the wave's column, two 16x16 halves.
      u4 a[kUA];
      lds_read_1k<kUA>(a, sa);
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int kb = 0; kb < NK; ++kb)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bf8 ah = __builtin_bit_cast(bf8, a[h * NK + kb]);
            if constexpr (X3)
              o[t][h] = mfma3(ah, __builtin_bit_cast(bf8, a[2 * NK + h * NK + kb]), vb[t][kb],
                              vbl[t][kb], o[t][h]);
            else
              o[t][h] = mfma_bf16(ah, vb[t][kb], o[t][h]);
          }
    }
    u4 b[RT * kX];
    lds_read_1k<RT * kX>(b, sa + kUA * 1024);
    const int row0 = 32 * (ch0 + k) + 8 * lg;
    const bool tail = X3 && 32 * (ch0 + k) + 32 > p.m;  // wave-uniform
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      float x[8], d[8];
      if constexpr (X3) {
        const f4 m0 = __builtin_bit_cast(f4, c[t][0]), m1 = __builtin_bit_cast(f4, c[t][kX - 1]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          x[e] = m0[e];
          x[4 + e] = m1[e];
        }
      } else {
        unpack8(c[t][0], x);
      }
      if (tail) {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = row0 + e < p.m ? x[e] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if constexpr (kA) {
          const float a1 = o[t][e >> 2][e & 3];
          // M - S = Uo Vo^T + clip(M - Uo Vo^T, -lambda, lambda)
          d[e] = a1 + __builtin_amdgcn_fmed3f(x[e] - a1, -lam, lam);
        } else {
          d[e] = x[e];
        }
      }
      if constexpr (X3) {
        bf8 dh, dl;
        split8(d, dh, dl);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct)
          acc[t][ct] = mfma3(dh, dl, __builtin_bit_cast(bf8, b[ct]),
                             __builtin_bit_cast(bf8, b[RT + ct]), acc[t][ct]);
      } else {
        const bf8 dh = pack8(d);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct)
          acc[t][ct] = mfma_bf16(dh, __builtin_bit_cast(bf8, b[ct]), acc[t][ct]);
      }
    }
  };

  // Groups of loads: chunk g's copies, then its M loads; groups are issued
  // in chunk order, so at chunk k the kD - 1 newer groups may stay in
  // flight. Every wave runs the same count of iterations and barriers.
  constexpr int kInFlight = (kD - 1) * (kPerWave + kX * KT);
#pragma unroll
  for (int g = 0; g < kD; ++g) {
    copy_u(g);
    load_m(ring[g], g);
    __builtin_amdgcn_sched_barrier(0);
  }
  const int nkp = (nk + kD - 1) / kD * kD;
  for (int k0 = 0; k0 < nkp; k0 += kD) {
#pragma unroll
    for (int d = 0; d < kD; ++d) {
      const int k = k0 + d;
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(kInFlight));
      bare_barrier();
      __builtin_amdgcn_sched_barrier(0);
      copy_u(k + kD);  // into the stage every wave finished with at chunk k - 1
      __builtin_amdgcn_sched_barrier(0);
      if (k < nk) chunk(ring[d], k);
      __builtin_amdgcn_sched_barrier(0);
      load_m(ring[d], k + kD);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // Drain the copies of the chunks past the end before the LDS is reused;
  // then each tile's partial W (red: KT blocks of kVStreamCols x RP).
  __syncthreads();
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        red[kVStreamCols * t + 16 * w + 4 * lg + v][16 * ct + li] = acc[t][ct][v];
  __syncthreads();
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    if (!valid[t]) continue;  // work-group-uniform
    const VTile& vt = p.vg64[gx0 + t];
    GLOBAL float* wp = gptr_w(p.Wpart) + ((int64_t)gy * p.NVP + vt.cl.vrow0 + vt.j0) * RP;
    for (int e = tid; e < kVStreamCols * RP; e += blockDim.x)
      wp[e] = red[kVStreamCols * t + e / RP][e % RP];
  }
}

// Work-group roles and tiles as in k_vpass (Q: persistent launch over the
// tile queue). KT > 0: the U operands staged in LDS, KT tiles per
// work-group (vpass_h3_tile; always in three-product rounds, picked by the
// column-group knob = 1 in one-product rounds); KT = 0, the one-product
// register form (vpass_h_tile).
template <int RT, int NK, int MODE, bool X3, bool Q, int KT>
__global__ __launch_bounds__(256) void k_vpass_h(DevParams p, const float* __restrict__ Ubase,
                                                 const float* __restrict__ Uold,
                                                 const float* __restrict__ Vold,
                                                 double* __restrict__ fin_Ginv, int fin) {
  constexpr bool ST = KT > 0;
  static_assert(ST || !X3, "three-product rounds run the staged form");
  // One LDS pool for both roles (sized for this rank, not the largest).
  constexpr int RP = 16 * RT;
  constexpr int kPool = vpass_pool_doubles(RP);
  constexpr int kStages = ST ? kLdsStages * vpass_h3_stage_bytes<RT, NK, MODE, X3>() / 8 : 0;
  constexpr int kRed = KT * kVStreamCols * RP / 2;  // every tile's W
  constexpr int kStaged = kStages > kRed ? kStages : kRed;
  __shared__ double pool[kPool > kStaged ? kPool : kStaged];
  float(*red)[RP] = reinterpret_cast<float(*)[RP]>(pool);
  auto run = [&](int t) {
    if constexpr (ST)
      vpass_h3_tile<RT, NK, MODE, X3, KT>(p, Ubase, Uold, Vold, t, red, pool);
    else
      vpass_h_tile<RT, NK, MODE>(p, Ubase, Uold, Vold, t, red);
  };
  if constexpr (!Q) {
    if (fin && blockIdx.x < 2) {
      finalize_role(p, fin_Ginv, (int)blockIdx.x, pool);
      return;
    }
    run((int)blockIdx.x - (fin ? 2 : 0));
  } else {
    if (fin && blockIdx.x < 2) finalize_role(p, fin_Ginv, (int)blockIdx.x, pool);
    const int ntiles = (ST ? vpass_h3_groups(p.ng64, KT) : p.ng64) * p.vsplit;
    for (int t = queue_next(p.queue, ntiles); t < ntiles; t = queue_next(p.queue, ntiles)) run(t);
  }
}

// Epilogue of a BF16 S-pass tile, after its P (ptile: the 128 rows' Lambda V,
// FP32) and the FP32 copy of A_i (fal, rows padded to kFS floats) are in LDS
// and visible to every wave: the U-step term of these 128 rows, then the
// tile's statistics.
template <int RT>
__device__ __forceinline__ void spass_h_finish(const DevParams& p, const float* __restrict__ U,
                                               int b, const ClientDev& cl,
                                               const float (*ptile)[16 * RT + 1],
                                               const float* fal, double sl2, double sl1,
                                               uint32_t nnz, double shb) {
  constexpr int RP = 16 * RT;
  constexpr int kFS = 16 * ((RP / 16) | 1);
  const int ci = cl.idx;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int MP = p.MP;
  const bool closed = p.u_mode != 0;
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

// ---------------------------------------------------------------------------
// BF16 S-pass: same grid (128-row blocks x clients, widest client first) and
// outputs as k_spass, over 32-column chunks, with 256 threads. Each wave
// takes four 16-row tiles, which share each chunk's V operands in registers,
// and every other chunk of its row group (two column phases). MFMA 1 forms
// (U V^T)^T for two 16x16 tiles per row tile with V's hP halves as A and U's
// hA as B, leaving lane l row l%16 and the eight columns 8 (l/16) + e of the
// chunk -- the lane's 16-byte load of the S-pass copy of M, and the A
// operand of MFMA 2 (P += Lambda V with V's hB packing as B). The phases'
// partial P are added in LDS in phase order. LDS holds P and an FP32 copy of
// A_i (54 KB at r = 64), so two work-groups fit on a compute unit and one's
// epilogue overlaps the other's sweep.
// ---------------------------------------------------------------------------
// HUB: 0, the Huber sum at the target lambda is left out (rounds at the
// target lambda); 1, it is taken; 2, p.huber decides per round (the test is
// if-converted, so its arithmetic runs on every entry).
template <int RT, int NK, int HUB>
__device__ __forceinline__ void spass_h_tile(const DevParams& p, const float* __restrict__ U, int b,
                                             int yi) {
  constexpr int RP = 16 * RT;
  constexpr int kRT = 4;        // 16-row tiles per wave
  constexpr int kPh = 2;        // column phases
  constexpr int kRG = 4 / kPh;  // row groups of 16 kRT rows
  static_assert(kRG * 16 * kRT == kSRows, "row groups cover the work-group's rows");
  const ClientDev cl = p.clients_lpt[yi];
  const int ci = cl.idx;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rg = wv % kRG, phase = wv / kRG;
  const int li = lane & 15, lg = lane >> 4;
  const int arow0 = b * kSRows + rg * 16 * kRT;
  const int MP = p.MP;

  bf8 ub[kRT][NK];  // MFMA 1 B operand: U[row][rank 32 kb + 8 (l/16) + e]
  {
    const GLOBAL bf8* UhA = reinterpret_cast<const GLOBAL bf8*>(gptr(u_hb(U, p)));
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb)
        ub[rt][kb] = UhA[((int64_t)((arow0 >> 4) + rt) * NK + kb) * 64 + lane];
    // Negated once: MFMA 1 then accumulates M - U V^T onto M (the residual
    // needs no subtraction per entry; the pass is VALU-bound).
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb)
        ub[rt][kb] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4, ub[rt][kb]) ^ 0x80008000u);
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
  if (p.u_mode != 0) {
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
  // Operands of one 32-column chunk, M (from HBM) and the V operands (from
  // L2) in the same ring slot, kept two chunks ahead. Single V buffers,
  // refilled right after their last use, left the L2 latency of every chunk
  // exposed (S-pass 1.12 -> 1.82 ms at 20000 x 100000, r = 64).
  struct MChunk {
    u4 m[kRT];  // M[row arow0 + 16 rt + l%16][col 32 cc + 8 (l/16) + e]
  };
  struct OpA {
    bf8 va[2][NK];  // V hP halves
  };
  struct OpB {
    bf8 vb[RT];  // V hB
  };
  constexpr int kDepth = 2;
  MChunk ring[kDepth];
  OpA oa[kDepth];
  OpB ob[kDepth];
  const int nch = (cl.n + 31) >> 5;
  const int nk = (nch - phase + kPh - 1) / kPh;  // chunks phase, phase + kPh, ... below nch
  auto load_m = [&](MChunk& c, int k) {
    const int cc = phase + kPh * k;
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) c.m[rt] = Ms[((int64_t)rt * nvc32 + cc) * 64];
  };
  auto load_a = [&](OpA& c, int k) {
    const int64_t vch = (cl.vrow0 >> 5) + phase + kPh * k;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) c.va[t][kb] = VhP[((vch * 2 + t) * NK + kb) * 64 + lane];
  };
  auto load_b = [&](OpB& c, int k) {
    const int64_t vch = (cl.vrow0 >> 5) + phase + kPh * k;
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) c.vb[ct] = VhB[(vch * RT + ct) * 64 + lane];
  };
  // Per row tile: MFMA 1, the residual's transpose M^T - (U V^T)^T in two
  // 16x16 halves, the accumulators starting from the lane's entries of M
  // (rows 8 (l/16) + e of the chunk's columns) and the U operand negated;
  // then the soft-threshold and statistics, then MFMA 2. Only one tile's
  // (U V^T)^T is live at a time.
  auto threshold_mfma2 = [&](const MChunk& c, const OpA& oa, const OpB& ob) {
    float l2 = 0.f, l1 = 0.f, hb = 0.f;
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      f4 o[2];
      {
        float x[8];
        unpack8(c.m[rt], x);
        o[0] = f4{x[0], x[1], x[2], x[3]};
        o[1] = f4{x[4], x[5], x[6], x[7]};
      }
#pragma unroll
      for (int kb = 0; kb < NK; ++kb)
#pragma unroll
        for (int t = 0; t < 2; ++t) o[t] = mfma_bf16(oa.va[t][kb], ub[rt][kb], o[t]);
      float lamv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float R = o[e >> 2][e & 3];
        const float L = __builtin_amdgcn_fmed3f(R, -lam, lam);  // clip(R, -lam, lam)
        const float Sv = R - L;
        lamv[e] = L;
        l2 = fmaf(L, L, l2);
        l1 += fabsf(Sv);
        if constexpr (HUB == 1) hb += huber1(R, lt);
        if constexpr (HUB == 2) if (hub) hb += huber1(R, lt);
        nnz += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(Sv != 0.f));
      }
      const bf8 lh = pack8(lamv);
#pragma unroll
      for (int ct = 0; ct < RT; ++ct) accp[rt][ct] = mfma_bf16(lh, ob.vb[ct], accp[rt][ct]);
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
        if (k < nk) threshold_mfma2(ring[d], oa[d], ob[d]);  // wave-uniform
        __builtin_amdgcn_sched_barrier(0);
        const int kn = min(k + kDepth, nk - 1);
        load_m(ring[d], kn);
        load_a(oa[d], kn);
        load_b(ob[d], kn);
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
  spass_h_finish<RT>(p, U, b, cl, ptile, fal, sl2, sl1, nnz, shb);
}

// ---------------------------------------------------------------------------
// BF16 S-pass with the V operands staged in LDS (three-product rounds
// always; one-product rounds with one S-pass phase), the V-pass's scheme with
// the roles of U and V exchanged. The four waves take 32 rows each (two
// 16-row tiles) and every 32-column chunk of the client, so a chunk's V
// operands (hP halves for MFMA 1, hB for MFMA 2; hi, and lo in three-product
// rounds) are the same for all of them: the waves copy them from L2 into
// LDS, kSpStages - 1 chunks ahead, beside the chunk's M loads (16 FP32 loads
// or 2 BF16 loads per wave), and each wave reads them from LDS at its use.
// S per entry is computed as in the register form; P sums a row's chunks in
// chunk order in one accumulator (the one-product register form adds two
// column phases' partial sums at the end).
// ---------------------------------------------------------------------------
constexpr int kSpStages = 3;
template <int RT, int NK, bool X3>
constexpr int spass_h3_units() {
  return (2 * NK + RT) * (X3 ? 2 : 1);
}
template <int RT, int NK, bool X3>
constexpr int spass_h3_stage_bytes() {
  return (spass_h3_units<RT, NK, X3>() + 3) / 4 * 4 * 1024;
}

template <int RT, int NK, int HUB, bool X3>
__device__ __forceinline__ void spass_h3_tile(const DevParams& p, const float* __restrict__ U, int b,
                                              int yi) {
  constexpr int RP = 16 * RT;
  constexpr int kRT = 2;  // 16-row tiles per wave
  static_assert(4 * 16 * kRT == kSRows, "four waves cover the work-group's rows");
  constexpr int kX = X3 ? 2 : 1;  // hi, and lo in three-product rounds
  constexpr int kVA = 2 * NK * kX;  // 1 KiB units of V's hP halves, then of V's hB
  constexpr int kUnits = spass_h3_units<RT, NK, X3>();
  constexpr int kPerWave = (kUnits + 3) / 4;
  constexpr int kStage = spass_h3_stage_bytes<RT, NK, X3>();
  static_assert(kStage == 4 * kPerWave * 1024, "one padded unit per wave and copy");
  constexpr int kD = kSpStages - 1;  // chunks ahead (M ring depth)
  const ClientDev cl = p.clients_lpt[yi];
  const int ci = cl.idx;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int arow0 = b * kSRows + 32 * wv;
  const int MP = p.MP;

  const int64_t uhl = hb_elems(MP, p.RK, p.RP) / 8, vhl = hb_elems(p.NVP, p.RK, p.RP) / 8;
  // MFMA 1 B operand (hi, lo): U[row][rank 32 kb + 8 (l/16) + e]
  bf8 ub[kRT][NK], ubl[X3 ? kRT : 1][NK];
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
    // Negated once: MFMA 1 then accumulates M - U V^T onto M.
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

  // A_i in FP32 for the epilogue, as in spass_h_tile; the staging buffers
  // and then P share one LDS block.
  constexpr int kFS = 16 * ((RP / 16) | 1);
  __shared__ float fal[RP * kFS];
  constexpr int kPBytes = kSRows * (RP + 1) * 4;  // P after the sweep
  constexpr int kSBytes = kSpStages * kStage;
  __shared__ float4 spool[(kPBytes > kSBytes ? kPBytes : kSBytes) / 16];
  float(*ptile)[RP + 1] = reinterpret_cast<float(*)[RP + 1]>(spool);
  if (p.u_mode != 0) {
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
  // M: (X3) the caller's FP32 block, one buffer resource per chunk (base at
  // its first column), fixed per-lane offsets; columns past n_i are out of
  // range and rows past m get an offset beyond any range, so both read 0.
  // Otherwise the S-pass BF16 copy of M, one 16-byte load per lane and row
  // tile (zero past m and n_i).
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
  const int nvc32 = (cl.n + kVPad - 1) / kVPad * (kVPad / 32);
  const GLOBAL u4* Ms = reinterpret_cast<const GLOBAL u4*>(gptr(p.Mbs)) +
                        (int64_t)cl.vrow0 * MP / 8 + (int64_t)(arow0 >> 4) * nvc32 * 64 + lane;
  const int nk = (cl.n + 31) >> 5;  // chunks (the same for every wave)

  // Units this wave copies (u = wv, wv + 4, ...; past the last: the last
  // again, into padding slots): source of chunk 0 and stride between chunks
  // in 16-byte elements. Unit u of a stage is the operand read at
  // stage + 1024 u + 16 lane.
  const GLOBAL bf8* src[kPerWave];
  int cstr[kPerWave];
#pragma unroll
  for (int i = 0; i < kPerWave; ++i) {
    const int u = min(wv + 4 * i, kUnits - 1);
    if (u < 2 * NK) {
      src[i] = VhP + u * 64 + lane;
      cstr[i] = 2 * NK * 64;
    } else if (u < kVA) {
      src[i] = VhP + vhl + (u - 2 * NK) * 64 + lane;
      cstr[i] = 2 * NK * 64;
    } else if (u < kVA + RT) {
      src[i] = VhB + (u - kVA) * 64 + lane;
      cstr[i] = RT * 64;
    } else {
      src[i] = VhB + vhl + (u - kVA - RT) * 64 + lane;
      cstr[i] = RT * 64;
    }
  }
  char* const stages = reinterpret_cast<char*>(spool);
  const uint32_t stage_lds = lds_addr(spool) + 16u * (uint32_t)lane;
  const int vch0 = cl.vrow0 >> 5;
  auto copy_v = [&](int k) {
    const int vch = vch0 + min(k, nk - 1);
    char* st = stages + (k % kSpStages) * kStage;
#pragma unroll
    for (int i = 0; i < kPerWave; ++i)
      __builtin_amdgcn_global_load_lds((GLOBAL void*)(src[i] + (int64_t)vch * cstr[i]),
                                       (lds_void*)(st + (wv + 4 * i) * 1024), 16, 0, 0);
  };
  struct MChunk {
    float mf[X3 ? kRT : 1][8];  // M[row arow0 + 16 rt + l%16][col 32 cc + 8 (l/16) + e]
    u4 m[X3 ? 1 : kRT];         // the same entries in BF16
  };
  MChunk ring[kD];
  auto load_m = [&](MChunk& c, int k) {
    const int cc = min(k, nk - 1);
    if constexpr (X3) {
      const rsrc_t rM =
          uniform_rsrc(cl.M + (int64_t)32 * cc * cl.ldm, chunk_bytes_from(cl.n, 32 * cc, cl.ldm));
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
        for (int e = 0; e < 8; ++e) c.mf[rt][e] = bload(rM, vm[rt][e], 0);
    } else {
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt) c.m[rt] = Ms[((int64_t)rt * nvc32 + cc) * 64];
    }
  };
  auto chunk = [&](const MChunk& c, int k) {
    const uint32_t sa = stage_lds + (uint32_t)((k % kSpStages) * kStage);
    // MFMA 1 for both row tiles: M^T - (U V^T)^T in two 16x16 halves per
    // tile, starting from the lane's entries of M.
    f4 o[kRT][2];
    {
      u4 a[kVA];
      lds_read_1k<kVA>(a, sa);
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt) {
        float x[8];
        if constexpr (X3) {
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = c.mf[rt][e];
        } else {
          unpack8(c.m[rt], x);
        }
        o[rt][0] = f4{x[0], x[1], x[2], x[3]};
        o[rt][1] = f4{x[4], x[5], x[6], x[7]};
#pragma unroll
        for (int kb = 0; kb < NK; ++kb)
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const bf8 ah = __builtin_bit_cast(bf8, a[t * NK + kb]);
            if constexpr (X3)
              o[rt][t] = mfma3(ah, __builtin_bit_cast(bf8, a[2 * NK + t * NK + kb]), ub[rt][kb],
                               ubl[rt][kb], o[rt][t]);
            else
              o[rt][t] = mfma_bf16(ah, ub[rt][kb], o[rt][t]);
          }
      }
    }
    u4 vb[RT * kX];
    lds_read_1k<RT * kX>(vb, sa + kVA * 1024);
    // Residual, soft-threshold and statistics per row tile, then MFMA 2.
    float l2 = 0.f, l1 = 0.f, hb = 0.f;
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
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
        for (int ct = 0; ct < RT; ++ct)
          accp[rt][ct] = mfma3(lh, ll, __builtin_bit_cast(bf8, vb[ct]),
                               __builtin_bit_cast(bf8, vb[RT + ct]), accp[rt][ct]);
      } else {
        const bf8 lh = pack8(lamv);
#pragma unroll
        for (int ct = 0; ct < RT; ++ct)
          accp[rt][ct] = mfma_bf16(lh, __builtin_bit_cast(bf8, vb[ct]), accp[rt][ct]);
      }
    }
    sl2 += (double)l2;
    sl1 += (double)l1;
    shb += (double)hb;
  };

  // Groups of loads: chunk g's copies, then its M loads, in chunk order; at
  // chunk k the kD - 1 newer groups may stay in flight. Every wave runs the
  // same count of iterations and barriers.
  constexpr int kInFlight = (kD - 1) * (kPerWave + (X3 ? 8 : 1) * kRT);
#pragma unroll
  for (int g = 0; g < kD; ++g) {
    copy_v(g);
    load_m(ring[g], g);
    __builtin_amdgcn_sched_barrier(0);
  }
  const int nkp = (nk + kD - 1) / kD * kD;
  for (int k0 = 0; k0 < nkp; k0 += kD) {
#pragma unroll
    for (int d = 0; d < kD; ++d) {
      const int k = k0 + d;
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(kInFlight));
      bare_barrier();
      __builtin_amdgcn_sched_barrier(0);
      copy_v(k + kD);  // into the stage every wave finished with at chunk k - 1
      __builtin_amdgcn_sched_barrier(0);
      if (k < nk) chunk(ring[d], k);
      __builtin_amdgcn_sched_barrier(0);
      load_m(ring[d], k + kD);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // Drain the copies past the end, then P of the four row groups.
  __syncthreads();
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) ptile[32 * wv + 16 * rt + 4 * lg + v][16 * ct + li] = accp[rt][ct][v];
  __syncthreads();
  spass_h_finish<RT>(p, U, b, cl, ptile, fal, sl2, sl1, nnz, shb);
}

// One work-group per tile (grid = row blocks x clients), or (Q) a persistent
// launch over the tile queue, tiles as in k_spass.
// The per-tile form asks for two work-groups per compute unit (the LDS
// allows it): at most 256 registers per lane, which it fits without spilling,
// so that one work-group's epilogue overlaps the other's sweep. The queue
// form's loop needs more registers and keeps the default bound.
// The per-tile form comes in two instantiations, with and without the Huber
// sum, picked at launch; the queue form decides per round.
// ST: the V operands staged in LDS (spass_h3_tile; always in three-product
// rounds, picked by one S-pass phase in one-product rounds), else the
// one-product register form (spass_h_tile).
template <int RT, int NK, bool X3, int HUB, bool ST>
__global__ __launch_bounds__(256, 2) void k_spass_h_tile(DevParams p, const float* __restrict__ U) {
  static_assert(ST || !X3, "three-product rounds run the staged form");
  if constexpr (ST)
    spass_h3_tile<RT, NK, HUB, X3>(p, U, (int)blockIdx.x, (int)blockIdx.y);
  else
    spass_h_tile<RT, NK, HUB>(p, U, (int)blockIdx.x, (int)blockIdx.y);
}
template <int RT, int NK, bool X3, bool ST>
__global__ __launch_bounds__(256) void k_spass_h_queue(DevParams p, const float* __restrict__ U) {
  static_assert(ST || !X3, "three-product rounds run the staged form");
  const int ntiles = p.nrb * p.E;
  for (int t = queue_next(p.queue + 2, ntiles); t < ntiles; t = queue_next(p.queue + 2, ntiles)) {
    if constexpr (ST)
      spass_h3_tile<RT, NK, 2, X3>(p, U, t % p.nrb, t / p.nrb);
    else
      spass_h_tile<RT, NK, 2>(p, U, t % p.nrb, t / p.nrb);
  }
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
  // Tiles per work-group of the staged form (0: the register form).
  const int kt = x3 ? (p.vcols == 1 ? 1 : 2) : (p.vcols == 1 ? 4 : 0);
  const int ntiles = (kt ? vpass_h3_groups(p.ng64, kt) : p.ng64) * p.vsplit;
  // The first round (S = 0) always runs one work-group per tile (group).
  auto go = [&](auto m, auto x, auto ktc) {
    constexpr int kMode = decltype(m)::value;
    constexpr bool kX3 = decltype(x)::value;
    constexpr int kKT = decltype(ktc)::value;
    if (kMode == kSRecompute && p.vqueue) {
      auto kernel = k_vpass_h<RT, NK, kSRecompute, kX3, true, kKT>;
      const int groups = pass_groups(kernel, 256, ntiles, 1);
      hipLaunchKernelGGL(kernel, dim3((unsigned)(groups + 2 * fin)), dim3(256), 0, st, p, U, Uold,
                         Vold, fin_Ginv, fin);
    } else {
      hipLaunchKernelGGL((k_vpass_h<RT, NK, kMode, kX3, false, kKT>),
                         dim3((unsigned)(ntiles + 2 * fin)), dim3(256), 0, st, p, U, Uold, Vold,
                         fin_Ginv, fin);
    }
  };
  using Z = std::integral_constant<int, kSZero>;
  using R = std::integral_constant<int, kSRecompute>;
  using F = std::false_type;
  using T = std::true_type;
  using K0 = std::integral_constant<int, 0>;
  using K1 = std::integral_constant<int, 1>;
  using K2 = std::integral_constant<int, 2>;
  using K4 = std::integral_constant<int, 4>;
  const bool rec = mode == kSRecompute;
  switch (kt) {
    case 1: rec ? go(R{}, T{}, K1{}) : go(Z{}, T{}, K1{}); break;
    case 2: rec ? go(R{}, T{}, K2{}) : go(Z{}, T{}, K2{}); break;
    case 4: rec ? go(R{}, F{}, K4{}) : go(Z{}, F{}, K4{}); break;
    default: rec ? go(R{}, F{}, K0{}) : go(Z{}, F{}, K0{}); break;
  }
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
    go(k_spass_h_queue<RT, NK, true, true>, k_spass_h_tile<RT, NK, true, 0, true>,
       k_spass_h_tile<RT, NK, true, 1, true>);
  else if (p.sphases == 1)
    go(k_spass_h_queue<RT, NK, false, true>, k_spass_h_tile<RT, NK, false, 0, true>,
       k_spass_h_tile<RT, NK, false, 1, true>);
  else
    go(k_spass_h_queue<RT, NK, false, false>, k_spass_h_tile<RT, NK, false, 0, false>,
       k_spass_h_tile<RT, NK, false, 1, false>);
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
