// The r x r and m x r kernels of a round (V finish, client factors, U update,
// finalize) and the small kernels behind the C ABI's outputs.
#include "rpca_device.h"

namespace rpca {

// ---------------------------------------------------------------------------
// V-pass, finalize: one work-group per 32 columns. W = sum of the row-split
// partials (fixed order, FP64), V = W (U^T U + rho I)^{-1} (eq. "condition1"),
// rounded to FP32 once and written in both layouts, plus the partial V^T V of
// these columns and its trace (the group's share of ||V||_F^2).
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_vfinal(DevParams p, const double* __restrict__ Gbase,
                                                int64_t g_stride, int rec) {
  constexpr int RP = 16 * RT;
  // rec = 1: record the previous round, whose finalize ran in the V-pass.
  if (rec && blockIdx.x == 0 && threadIdx.x == 0) {
    double st[7];
    for (int q = 0; q < 7; ++q) st[q] = p.stat_part[q];
    fin_record(p, st, p.dstate->u_sq_next);
  }
  // G^{-1} is staged in LDS kKB rows at a time: all of it up to four rank
  // tiles, half of it beyond (the whole of it and W would not fit the LDS at
  // r = 128); the products still run over k in increasing order.
  constexpr int kKB = RT <= 4 ? RP : RP / 2;
  __shared__ double wd[kVCols][RP + 1];
  __shared__ double gl[kKB * RP];
  const VGroup vg = p.vgroups[blockIdx.x];
  const double* __restrict__ Gi = Gbase + (int64_t)vg.client * g_stride;
  const int tid = threadIdx.x;
  const int vrow = vg.vrow;
  const int64_t split_stride = (int64_t)p.NVP * RP;
  constexpr int kPer = (kVCols * RP + 255) / 256;
  constexpr int kGPer = (kKB * RP + 255) / 256;
  {
    // All of a thread's loads (kWB row splits of each of its W entries, and
    // its share of G^{-1}'s first kKB rows) are issued before any is used;
    // splits are summed in increasing order. Wider ranks batch fewer splits,
    // which keeps the batch's addresses within the register file.
    double gv_[kGPer];
#pragma unroll
    for (int q = 0; q < kGPer; ++q) {
      const int e = tid + q * 256;
      gv_[q] = Gi[e];  // e < RP^2: a multiple of 256 is read, kKB RP kept
    }
    double acc[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
    constexpr int kWB = RT <= 2 ? 8 : RT <= 4 ? 4 : 2;
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
      if (e < kKB * RP) gl[e] = gv_[q];
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
    for (int kb = 0; kb < RP; kb += kKB) {
      if (kb > 0) {  // (wide ranks) the next kKB rows of G^{-1}
        __syncthreads();
        for (int e = tid; e < kKB * RP; e += 256) gl[e] = Gi[(int64_t)kb * RP + e];
        __syncthreads();
      }
      const int kend = min(p.r, kb + kKB);
#pragma unroll 2
      for (int k = kb; k < kend; ++k) {
        const double* gk = gl + (k - kb) * RP;
        if constexpr (256 % RP == 0) {
          const double g = gk[tid % RP];
#pragma unroll
          for (int q = 0; q < kPer; ++q) sv[q] += wd[(tid + 256 * q) / RP][k] * g;
        } else {
#pragma unroll
          for (int q = 0; q < kPer; ++q) {
            const int e = tid + 256 * q;
            sv[q] += wd[e / RP][k] * gk[e % RP];
          }
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
  // (Beyond four rank tiles the block's rows go in sweeps of four, which
  // keeps its sums within the registers; same sums.) The threads on the
  // diagonal (ta = tb) add their diagonal entries in rank order for the trace.
  // Only the lower triangle is written: the partial is symmetric bit for bit
  // (each entry multiplies the same two factors both ways round), and
  // k_client_factor reads entry (a, b) with a >= b.
  double* gv = p.gv_part + (int64_t)blockIdx.x * RP * RP;
  constexpr int kXB = RT <= 4 ? RT : 4;
  const bool on_diag = (tid >> 4) == (tid & 15);
  const bool lower = (tid >> 4) >= (tid & 15);
  double dtr = 0.0;
#pragma unroll
  for (int x0 = 0; x0 < RT; x0 += kXB) {
    if (!lower) break;
    const int a0 = RT * (tid >> 4) + x0, b0 = RT * (tid & 15);
    double sg[kXB][RT];
#pragma unroll
    for (int x = 0; x < kXB; ++x)
#pragma unroll
      for (int y = 0; y < RT; ++y) sg[x][y] = 0.0;
#pragma unroll 2
    for (int j = 0; j < kVCols; ++j) {
      double va[kXB], vb[RT];
#pragma unroll
      for (int x = 0; x < kXB; ++x) va[x] = x0 + x < RT ? wd[j][a0 + x] : 0.0;
#pragma unroll
      for (int y = 0; y < RT; ++y) vb[y] = wd[j][b0 + y];
#pragma unroll
      for (int x = 0; x < kXB; ++x)
#pragma unroll
        for (int y = 0; y < RT; ++y) sg[x][y] += va[x] * vb[y];
    }
#pragma unroll
    for (int x = 0; x < kXB; ++x)
      if (x0 + x < RT) {
#pragma unroll
        for (int y = 0; y < RT; ++y)
          if (a0 + x >= b0 + y) gv[(a0 + x) * RP + b0 + y] = sg[x][y];
        if (on_diag) dtr += sg[x][x0 + x];
      }
  }
  __shared__ double trs[16];
  if (on_diag) trs[tid >> 4] = dtr;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += trs[k];
    p.gv_tr[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Per-client r x r factor for the closed-form U step:
//   A_i = (V_i^T V_i + c_i I)^{-1},  c_i = rho n_i / n.
// (The step's other factor, V_i^T V_i A_i, is I - c_i A_i, which the S-pass
// epilogue applies as U_i + (P - c_i U_i) A_i.) One work-group per client;
// FP64 throughout.
// ---------------------------------------------------------------------------
// Threads of a client-factor work-group.
constexpr int cf_threads(int) { return 1024; }
template <int RT>
__global__ __launch_bounds__(cf_threads(RT)) void k_client_factor(DevParams p) {
  constexpr int RP = 16 * RT, NT = cf_threads(RT);
  // Lower-triangle entries per thread: three up to r = 64 (1024 x 3 >= 64 x
  // 65 / 2), nine at r = 128.
  constexpr int kCE = RT <= 4 ? 3 : (RP * (RP + 1) / 2 + NT - 1) / NT;
  __shared__ double A[RP * RP];
  const int r = p.r;
  const int64_t RR = (int64_t)RP * RP;
  const ClientDev cl = p.clients[blockIdx.x];
  const int tid = threadIdx.x;
  if (cl.g1 - cl.g0 <= 16) {
    // One block of groups: one batch of loads per entry; the partials hold
    // the lower triangle, so (a, b) reads (max, min).
    for (int e = tid; e < r * r; e += blockDim.x) {
      const int a = e / r, b = e % r;
      const int hi = a > b ? a : b, lo = a > b ? b : a;
      const double s = sum_strided(p.gv_part + (int64_t)cl.g0 * RR + hi * RP + lo, cl.g1 - cl.g0, RR);
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
    const int nl = r * (r + 1) / 2, ng = cl.g1 - cl.g0;
    const double* __restrict__ gp = p.gv_part + (int64_t)cl.g0 * RR;
    int ia[kCE], ib[kCE];
    double s[kCE];
#pragma unroll
    for (int q = 0; q < kCE; ++q) {
      const int e = tid + q * NT;
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
    // (Beyond four rank tiles, with up to three times the entries per
    // thread, one group at a time: same sums.)
    constexpr int kGB = RT <= 4 ? 8 : 1;
    for (int g0 = 0; g0 < ng; g0 += 16) {
      double t[kCE];
#pragma unroll
      for (int q = 0; q < kCE; ++q) t[q] = 0.0;
#pragma unroll
      for (int h = 0; h < 16; h += kGB) {
        double v[kCE][kGB];
#pragma unroll
        for (int q = 0; q < kCE; ++q)
#pragma unroll
          for (int u = 0; u < kGB; ++u) {
            const int g = g0 + h + u;
            const double x = gp[(int64_t)min(g, ng - 1) * RR + max(ia[q], 0) * RP + ib[q]];
            v[q][u] = x * (double)(ia[q] >= 0 && g < ng);
          }
#pragma unroll
        for (int q = 0; q < kCE; ++q)
#pragma unroll
          for (int u = 0; u < kGB; ++u) t[q] += v[q][u];
      }
#pragma unroll
      for (int q = 0; q < kCE; ++q) s[q] += t[q];
    }
#pragma unroll
    for (int q = 0; q < kCE; ++q)
      if (ia[q] >= 0) {
        const int a = ia[q], b = ib[q];
        A[a * r + b] = s[q] + (a == b ? cl.c : 0.0);
        A[b * r + a] = s[q] + (a == b ? cl.c : 0.0);
      }
  }
  __syncthreads();
  spd_inverse<kCE, true>(A, r, r);
  double* Af = p.Afac + (int64_t)blockIdx.x * RR;
  for (int e = tid; e < RR; e += blockDim.x) {
    const int a = e / RP, b = e % RP;
    Af[e] = a < r && b < r ? A[a * r + b] : 0.0;
  }
}


// Partial Gram of kURows rows held in LDS (FP64, row stride RP), by a
// 256-thread work-group: thread (ta, tb) = (tid / 16, tid % 16) forms the
// RT x RT block of entries (RT ta + x, RT tb + y), so each LDS read feeds RT
// FMAs (beyond four rank tiles, the block's rows x in sweeps of two, which
// keeps the sums within the registers). Every entry is summed as two chains,
// even rows and odd rows, each in row order, then added.
template <int RT>
__device__ void gram_rows_partial(const double* ul, double* out) {
  constexpr int RP = 16 * RT;
  constexpr int kXB = RT <= 4 ? RT : 2;
#pragma unroll
  for (int x0 = 0; x0 < RT; x0 += kXB) {
    const int a0 = RT * (threadIdx.x >> 4) + x0, b0 = RT * (threadIdx.x & 15);
    double s0[kXB][RT], s1[kXB][RT];
#pragma unroll
    for (int x = 0; x < kXB; ++x)
#pragma unroll
      for (int y = 0; y < RT; ++y) s0[x][y] = s1[x][y] = 0.0;
#pragma unroll 4
    for (int j = 0; j < kURows; j += 2) {
      double va0[kXB], vb0[RT], va1[kXB], vb1[RT];
#pragma unroll
      for (int x = 0; x < kXB; ++x) {
        va0[x] = x0 + x < RT ? ul[j * RP + a0 + x] : 0.0;
        va1[x] = x0 + x < RT ? ul[(j + 1) * RP + a0 + x] : 0.0;
      }
#pragma unroll
      for (int y = 0; y < RT; ++y) {
        vb0[y] = ul[j * RP + b0 + y];
        vb1[y] = ul[(j + 1) * RP + b0 + y];
      }
#pragma unroll
      for (int x = 0; x < kXB; ++x)
#pragma unroll
        for (int y = 0; y < RT; ++y) {
          s0[x][y] += va0[x] * vb0[y];
          s1[x][y] += va1[x] * vb1[y];
        }
    }
#pragma unroll
    for (int x = 0; x < kXB; ++x)
      if (x0 + x < RT)
#pragma unroll
        for (int y = 0; y < RT; ++y) out[(a0 + x) * RP + b0 + y] = s0[x][y] + s1[x][y];
  }
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
  __shared__ double ul[kURows * RP];
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
  constexpr int kUB = RT <= 2 ? 8 : RT <= 4 ? 4 : 2;
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
  // A step multiplier omega != 1 scales the consensus step: U^(t+1) = U^(t) +
  // omega (mean_i T_i - U^(t)) (for the gradient step, eta becomes omega eta).
  const bool relax = final_step && p.omega != 1.0;
  float* __restrict__ Uo = Uout + (final_step ? 0 : (int64_t)blockIdx.y * uout_stride);
  double dsq = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = cq + 4 * q;
    double x = acc[q] * scale;
    if (relax) x = (double)uprev[q] + p.omega * (x - (double)uprev[q]);
    const float v = (a < p.m && c < r) ? (float)x : 0.f;
    fb_store(Uo, MP, RP, p.NS, a, c, v);
    if (p.bf16) hb_store(u_hb(Uo, p), MP, p, a, c, v);
    ul[al * RP + c] = (double)v;
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
template <int RT>
__global__ __launch_bounds__(256) void k_gram_init(DevParams p, const float* __restrict__ U) {
  constexpr int RP = 16 * RT;
  __shared__ double ul[kURows * RP];
  for (int e = threadIdx.x; e < kURows * RP; e += blockDim.x) {
    const int al = e % kURows, c = e / kURows;
    ul[al * RP + c] = (double)U[(int64_t)c * p.MP + blockIdx.x * kURows + al];
  }
  __syncthreads();
  gram_rows_partial<RT>(ul, p.gram_part + (int64_t)blockIdx.x * RP * RP);
}


// Gram sums for the finalize at ranks above kFoldMaxRP: entry e < r^2 of
// slot blockIdx.y over the slot's row-block partials, in the order fin_gram
// sums them, into Ginv slot blockIdx.y (row stride r), which the finalize
// then reads and overwrites with the inverse. Spread over r^2 / 256
// work-groups per slot: the sums read nub r^2 doubles (16 MB at m = 8000,
// r = 128), which the finalize's one work-group would read at the latency
// of a single compute unit.
__global__ __launch_bounds__(256) void k_gram_sum(DevParams p, double* Ginv, int64_t g_stride) {
  const int gi = (int)blockIdx.y, e = (int)blockIdx.x * 256 + (int)threadIdx.x, r = p.r;
  if (e >= r * r) return;
  const int a = e / r, b = e - a * r;
  const int64_t RR = (int64_t)p.RP * p.RP;
  Ginv[(int64_t)gi * g_stride + e] =
      sum_strided(p.gram_part + (int64_t)gi * p.nub * RR + a * p.RP + b, p.nub, RR);
}

// Standalone finalize: one work-group of NT threads per Gram slot (grid =
// per_client ? E : 1), for ranks up to RMAX: 64 (Gram summed here), or 128
// (Gram summed by k_gram_sum into the slot; 1024 threads share the sweep).
template <int RMAX, int NT>
__global__ __launch_bounds__(NT) void k_finalize(DevParams p, double* Ginv, int64_t g_stride,
                                                 int per_client, int record) {
  __shared__ double A[RMAX * RMAX];
  __shared__ double st[7];
  const int gi = (int)blockIdx.x;
  if constexpr (RMAX > kFoldMaxRP) {
    const double* g = Ginv + (int64_t)gi * g_stride;
    for (int e = threadIdx.x; e < p.r * p.r; e += NT) A[e] = g[e];
  } else {
    fin_gram(p, gi, A);
  }
  if (record && !per_client) fin_stats(p, st);
  __syncthreads();
  constexpr int kEPT = (RMAX * (RMAX + 1) / 2 + NT - 1) / NT;
  const double tr = fin_inverse<kEPT, (RMAX > kFoldMaxRP || kEPT <= 4)>(p, A, Ginv, g_stride, gi);
  if (threadIdx.x != 0) return;
  if (per_client)
    p.ucl_sq[gi] = tr;
  else if (!record)
    p.dstate->u_sq = tr;
  else
    fin_record(p, st, tr);
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

// Output j >= 0 of SplitMix64 (Steele, Lea and Flood, 2014) seeded with
// `seed`, in counter form: the generator's state after j + 1 steps is
// seed + (j + 1) times the golden-ratio increment, and the output is the
// state's mix.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// U^(0) into a factor block, entry (a, c) = the Box-Muller normal of outputs
// 2k and 2k + 1, k = c m + a: sqrt(-2 ln(1 - u1)) cos(2 pi u2) with
// u = (x >> 11) 2^-53, in FP64, rounded to FP32 (zeros outside m x r).
__global__ void k_init_U_gauss(DevParams p, uint64_t seed, float* __restrict__ Ufb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)p.RP * p.MP) return;
  const int a = (int)(e % p.MP), c = (int)(e / p.MP);
  float v = 0.f;
  if (a < p.m && c < p.r) {
    const uint64_t k = (uint64_t)c * (uint64_t)p.m + (uint64_t)a;
    const double u1 = (double)(splitmix64_at(seed, 2 * k) >> 11) * 0x1.0p-53;
    const double u2 = (double)(splitmix64_at(seed, 2 * k + 1) >> 11) * 0x1.0p-53;
    v = (float)(sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586476925 * u2));
  }
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

// Partial cross-Gram matrices for ||X1 Y1^T - X2 Y2^T||_F^2 over widths up to
// W (64, or 128 beyond). Work-groups blockIdx.x in [0, NB) sweep the X side
// (MP rows), [NB, 2 NB) the Y side (NVP rows), 64 rows at a time; blockIdx.y
// takes a slice of kDistSlice of the 3 W^2 entries of [Z1^T Z1 | Z1^T Z2 |
// Z2^T Z2] (W x W FP64 each), 48 per thread in registers. part[blockIdx.x]
// holds the 3 W^2 entries; 2 NB 3 W^2 is kDistPartDoubles at both widths.
constexpr int kDistRows = 64;
template <int W>
__global__ __launch_bounds__(256) void k_dist_partial(DevParams p, const float* __restrict__ X1,
                                                      const float* __restrict__ Y1, int rp1,
                                                      const float* __restrict__ X2,
                                                      const float* __restrict__ Y2, int rp2,
                                                      double* __restrict__ part) {
  constexpr int NB = dist_blocks(W), ET = 3 * W * W;
  __shared__ float z1[kDistRows][W + 1];
  __shared__ float z2[kDistRows][W + 1];
  constexpr int kPer = kDistSlice / 256;
  const bool xside = (int)blockIdx.x < NB;
  const int blk = xside ? blockIdx.x : blockIdx.x - NB;
  const int ld = xside ? p.MP : p.NVP;
  const float* A = xside ? X1 : Y1;
  const float* B = xside ? X2 : Y2;
  const int e0 = (int)blockIdx.y * kDistSlice;
  double acc[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
  for (int row0 = blk * kDistRows; row0 < ld; row0 += NB * kDistRows) {
    __syncthreads();
    for (int e = threadIdx.x; e < kDistRows * W; e += blockDim.x) {
      const int j = e % kDistRows, c = e / kDistRows;
      const int row = row0 + j;
      z1[j][c] = (row < ld && c < rp1) ? A[(int64_t)c * ld + row] : 0.f;
      z2[j][c] = (row < ld && c < rp2) ? B[(int64_t)c * ld + row] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = e0 + threadIdx.x + q * 256;
      const int which = e / (W * W);
      const int a = (e / W) % W, b = e % W;
      const int ra = which == 2 ? rp2 : rp1;
      const int rb = which == 0 ? rp1 : rp2;
      if (a < ra && b < rb) {
        const float(*za)[W + 1] = which == 2 ? z2 : z1;
        const float(*zb)[W + 1] = which == 0 ? z1 : z2;
        double s = 0.0;
        for (int j = 0; j < kDistRows; ++j) s += (double)za[j][a] * (double)zb[j][b];
        acc[q] += s;
      }
    }
  }
  double* o = part + (int64_t)blockIdx.x * ET + e0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) o[threadIdx.x + q * 256] = acc[q];
}

// Level 1: 3 W^2 / 256 work-groups x 256 entries; each entry's X- and Y-side
// Grams are summed over the partials and multiplied; part2[blk] = block sum.
template <int W>
__global__ __launch_bounds__(256) void k_dist_reduce(const double* __restrict__ part,
                                                     double* __restrict__ part2) {
  constexpr int NB = dist_blocks(W), ET = 3 * W * W;
  __shared__ double red[4];
  const int e = blockIdx.x * 256 + threadIdx.x;
  double gx = 0.0, gy = 0.0;
  for (int k = 0; k < NB; ++k) gx += part[(int64_t)k * ET + e];
  for (int k = 0; k < NB; ++k) gy += part[(int64_t)(NB + k) * ET + e];
  double t = wave_sum(gx * gy);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) part2[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

template <int W>
__global__ void k_dist_final(const double* __restrict__ part2, double* __restrict__ out2) {
  if (threadIdx.x != 0) return;
  constexpr int per = (W * W) / 256;  // level-1 blocks per Gram pair
  double s[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 3 * per; ++k) s[k / per] += part2[k];
  out2[0] = s[0] - 2.0 * s[1] + s[2];
  out2[1] = s[2];
}

template <int RT>
static hipError_t launch_vfinal_t(const DevParams& p, const double* Ginv, int64_t g_stride,
                                  int rec, hipStream_t st) {
  hipLaunchKernelGGL(k_vfinal<RT>, dim3(p.ngroups), dim3(256), 0, st, p, Ginv, g_stride, rec);
  return hipGetLastError();
}

hipError_t launch_vfinal(const DevParams& p, const double* Ginv, int64_t g_stride, int rec,
                         hipStream_t st) {
  return with_rt(p.RP, [&](auto rt) {
    return launch_vfinal_t<decltype(rt)::value>(p, Ginv, g_stride, rec, st);
  });
}

hipError_t launch_client_factor(const DevParams& p, hipStream_t st) {
  return with_rt(p.RP, [&](auto rt) {
    constexpr int RT = decltype(rt)::value;
    hipLaunchKernelGGL(k_client_factor<RT>, dim3(p.E), dim3(cf_threads(RT)), 0, st, p);
    return hipGetLastError();
  });
}

hipError_t launch_uupdate(const DevParams& p, float* Uout, int64_t uout_stride,
                          const float* Uprev_cons, int final_step, hipStream_t st) {
  dim3 grid(p.nub, final_step ? 1 : p.E), block(256);
  return with_rt(p.RP, [&](auto rt) {
    hipLaunchKernelGGL(k_uupdate<decltype(rt)::value>, grid, block, 0, st, p, Uout, uout_stride,
                       Uprev_cons, final_step);
    return hipGetLastError();
  });
}

hipError_t launch_finalize(const DevParams& p, double* Ginv, int64_t g_stride, int per_client,
                           int record, hipStream_t st) {
  const int slots = per_client ? p.E : 1;
  if (p.RP <= kFoldMaxRP) {
    hipLaunchKernelGGL((k_finalize<kFoldMaxRP, kFinThreads>), dim3(slots), dim3(kFinThreads), 0,
                       st, p, Ginv, g_stride, per_client, record);
  } else {
    hipLaunchKernelGGL(k_gram_sum, dim3((p.r * p.r + 255) / 256, slots), dim3(256), 0, st, p,
                       Ginv, g_stride);
    hipLaunchKernelGGL((k_finalize<kMaxRank, 1024>), dim3(slots), dim3(1024), 0, st, p, Ginv,
                       g_stride, per_client, record);
  }
  return hipGetLastError();
}

hipError_t launch_gram_init(const DevParams& p, const float* U, hipStream_t st) {
  return with_rt(p.RP, [&](auto rt) {
    hipLaunchKernelGGL(k_gram_init<decltype(rt)::value>, dim3(p.nub), dim3(256), 0, st, p, U);
    return hipGetLastError();
  });
}

hipError_t launch_copy_in_U(const DevParams& p, const float* U0, int64_t ldu, float* Ufb,
                            hipStream_t st) {
  const int64_t tot = (int64_t)p.RP * p.MP;
  hipLaunchKernelGGL(k_copy_in_U, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p, U0,
                     ldu, Ufb);
  return hipGetLastError();
}

hipError_t launch_init_U_gauss(const DevParams& p, uint64_t seed, float* Ufb, hipStream_t st) {
  const int64_t tot = (int64_t)p.RP * p.MP;
  hipLaunchKernelGGL(k_init_U_gauss, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p,
                     seed, Ufb);
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

template <int W>
static hipError_t launch_distance_t(const DevParams& p, const float* X1, const float* Y1,
                                    int rp1, const float* X2, const float* Y2, int rp2,
                                    double* part, double* part2, double* out2, hipStream_t st) {
  constexpr int ET = 3 * W * W;
  hipLaunchKernelGGL(k_dist_partial<W>, dim3(2 * dist_blocks(W), ET / kDistSlice), dim3(256), 0,
                     st, p, X1, Y1, rp1, X2, Y2, rp2, part);
  hipLaunchKernelGGL(k_dist_reduce<W>, dim3(ET / 256), dim3(256), 0, st, part, part2);
  hipLaunchKernelGGL(k_dist_final<W>, dim3(1), dim3(64), 0, st, part2, out2);
  return hipGetLastError();
}

hipError_t launch_factor_distance(const DevParams& p, const float* X1, const float* Y1, int rp1,
                                  const float* X2, const float* Y2, int rp2, double* part,
                                  double* part2, double* out2, hipStream_t st) {
  if (rp1 < 1 || rp2 < 1 || rp1 > kMaxRank || rp2 > kMaxRank) return hipErrorInvalidValue;
  if (rp1 <= 64 && rp2 <= 64)
    return launch_distance_t<64>(p, X1, Y1, rp1, X2, Y2, rp2, part, part2, out2, st);
  return launch_distance_t<kMaxRank>(p, X1, Y1, rp1, X2, Y2, rp2, part, part2, out2, st);
}


}  // namespace rpca
