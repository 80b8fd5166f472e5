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
//   finalize : U^T U + rho I, its FP64 Cholesky factor and inverse, and the
//              round's FP64 statistics.
// The rank-r contractions run on the fp32 MFMA (v_mfma_f32_16x16x4f32); the
// r x r algebra and all reductions that feed a convergence test are FP64.
#include "rpca_internal.h"

#include <cmath>

namespace rpca {

typedef float f4 __attribute__((ext_vector_type(4)));

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

// In-place inverse of an r x r SPD matrix A (row stride ld, in LDS) through
// its Cholesky factor: A = L L^T, A^{-1} = L^{-T} L^{-1}. X is r x ld scratch.
// A non-positive pivot yields NaN, which the round statistics then expose.
__device__ void spd_inverse(double* A, double* X, int r, int ld) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < r; ++k) {
    if (tid == 0) {
      const double d = A[k * ld + k];
      A[k * ld + k] = d > 0.0 ? sqrt(d) : NAN;
    }
    __syncthreads();
    const double dk = A[k * ld + k];
    for (int i = k + 1 + tid; i < r; i += nt) A[i * ld + k] /= dk;
    __syncthreads();
    const int rem = r - k - 1;
    for (int e = tid; e < rem * rem; e += nt) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      if (j <= i) A[i * ld + j] -= A[i * ld + k] * A[j * ld + k];
    }
    __syncthreads();
  }
  for (int c = tid; c < r; c += nt) {  // column c of L^{-1}
    for (int i = 0; i < r; ++i) {
      if (i < c) {
        X[i * ld + c] = 0.0;
        continue;
      }
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= A[i * ld + k] * X[k * ld + c];
      X[i * ld + c] = s / A[i * ld + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int pq = e / r, qq = e % r;
    const int k0 = pq > qq ? pq : qq;
    double s = 0.0;
    for (int k = k0; k < r; ++k) s += X[k * ld + pq] * X[k * ld + qq];
    A[pq * ld + qq] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// V-pass: one work-group per (client, 32 columns); 8 waves split the rows.
// Wave tile: 16 rows x 16 columns of D = M - S per MFMA step. Lane l holds
// rows 4*(l/16)..+3 of column l%16 (one float4 along the contiguous rows), so
// element s of that float4 is the A operand of step s; U^T supplies the B
// operand as a float4 of U's column-major layout. Output W[col][c].
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(512) void k_vpass(DevParams p, const float* __restrict__ Ubase,
                                               int64_t u_stride, const double* __restrict__ Gbase,
                                               int64_t g_stride) {
  constexpr int RP = 16 * RT;
  __shared__ float red[kVWaves][kVCols][RP];
  __shared__ double wd[kVCols][RP + 1];
  const VGroup vg = p.vgroups[blockIdx.x];
  const ClientDev cl = p.clients[vg.client];
  const float* __restrict__ U = Ubase + (int64_t)vg.client * u_stride;
  const double* __restrict__ Gi = Gbase + (int64_t)vg.client * g_stride;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lg = lane >> 4;
  const float* __restrict__ Sblk = p.S + cl.s_off;

  f4 acc[2][RT];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) acc[t][ct] = f4{0.f, 0.f, 0.f, 0.f};

  const int nchunks = (p.m + 15) >> 4;
  for (int ch = w; ch < nchunks; ch += kVWaves) {
    const int row = (ch << 4) + 4 * lg;
    f4 d[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int col = vg.j0 + 16 * t + li;
      f4 dv = {0.f, 0.f, 0.f, 0.f};
      if (col < cl.n && row < p.m) {
        const f4 mv = *reinterpret_cast<const f4*>(cl.M + (int64_t)col * cl.ldm + row);
        const f4 sv = *reinterpret_cast<const f4*>(Sblk + (int64_t)col * p.lds + row);
        dv = mv - sv;
        if (row + 4 > p.m) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (row + e >= p.m) dv[e] = 0.f;
        }
      }
      d[t] = dv;
    }
    f4 u[RT];
#pragma unroll
    for (int ct = 0; ct < RT; ++ct)
      u[ct] = *reinterpret_cast<const f4*>(U + (int64_t)(16 * ct + li) * p.MP + row);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) acc[t][ct] = mfma4(d[t][s], u[ct][s], acc[t][ct]);
  }

#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w][16 * t + 4 * lg + v][16 * ct + li] = acc[t][ct][v];
  __syncthreads();
  for (int e = tid; e < kVCols * RP; e += blockDim.x) {
    const int j = e / RP, c = e % RP;
    double s = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < kVWaves; ++w2) s += (double)red[w2][j][c];
    wd[j][c] = s;
  }
  __syncthreads();
  double* gl = reinterpret_cast<double*>(&red[0][0][0]);  // RP*RP doubles fit
  for (int e = tid; e < RP * RP; e += blockDim.x) gl[e] = Gi[e];
  __syncthreads();

  // V[j][c] = sum_k W[j][k] Ginv[k][c], rounded to FP32 once.
  constexpr int kPer = (kVCols * RP + 511) / 512;
  float vres[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * 512;
    float vf = 0.f;
    if (e < kVCols * RP) {
      const int j = e / RP, c = e % RP;
      if (j < vg.ncols && c < p.r) {
        double s = 0.0;
        for (int k = 0; k < p.r; ++k) s += wd[j][k] * gl[k * RP + c];
        vf = (float)s;
      }
    }
    vres[q] = vf;
  }
  __syncthreads();
  const int vrow = cl.vrow0 + vg.j0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * 512;
    if (e < kVCols * RP) {
      const int j = e / RP, c = e % RP;
      wd[j][c] = (double)vres[q];
      p.Vrow[(int64_t)(vrow + j) * RP + c] = vres[q];
      p.Vcol[(int64_t)c * p.NVP + vrow + j] = vres[q];
    }
  }
  __syncthreads();
  double* gv = p.gv_part + (int64_t)blockIdx.x * RP * RP;
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    const int a = e / RP, b = e % RP;
    double s = 0.0;
    for (int j = 0; j < kVCols; ++j) s += wd[j][a] * wd[j][b];
    gv[e] = s;
  }
}

// ---------------------------------------------------------------------------
// Per-client r x r factors for the closed-form U step:
//   A_i = (V_i^T V_i + c_i I)^{-1},  B_i = V_i^T V_i A_i,  c_i = rho n_i / n.
// One work-group per client; FP64 throughout.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_client_factor(DevParams p) {
  // Static LDS (96 KiB at r = 64): gfx950 work-groups may hold up to 160 KiB.
  __shared__ double A[kMaxRank * kMaxRank], X[kMaxRank * kMaxRank], G[kMaxRank * kMaxRank];
  const int r = p.r, RP = p.RP;
  const ClientDev cl = p.clients[blockIdx.x];
  const int tid = threadIdx.x;
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int a = e / r, b = e % r;
    double s = 0.0;
    for (int g = cl.g0; g < cl.g1; ++g) s += p.gv_part[(int64_t)g * RP * RP + a * RP + b];
    G[e] = s;
    A[e] = s + (a == b ? cl.c : 0.0);
  }
  __syncthreads();
  spd_inverse(A, X, r, r);
  double* Af = p.Afac + (int64_t)blockIdx.x * RP * RP;
  double* Bf = p.Bfac + (int64_t)blockIdx.x * RP * RP;
  for (int e = tid; e < RP * RP; e += blockDim.x) {
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

// ---------------------------------------------------------------------------
// S-pass: one work-group per (128-row block, client); each of the 4 waves owns
// 32 rows (two 16-row tiles) and sweeps the client's columns 16 at a time.
// MFMA 1 forms (U V^T)^T for a 16x16 tile with V as the A operand and U^T as
// the B operand, so lane l ends up with row l%16 and columns 4*(l/16)+v.
// That is exactly the A-operand layout of MFMA 2 (P += Lambda V, contraction
// over columns), so Lambda goes from the accumulator to the next MFMA without
// any data movement. M is read and S written one dword per lane per column
// (16 consecutive rows per column per instruction).
// The contraction index of MFMA 1 is split as k-group g = l/16 taking rank
// indices g*NS + s, s < NS = ceil(r/4), so no padding steps run for r % 16.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_spass(DevParams p, const float* __restrict__ Ubase,
                                               int64_t u_stride) {
  constexpr int RP = 16 * RT, NSMAX = 4 * RT;
  const int b = blockIdx.x, ci = blockIdx.y;
  const ClientDev cl = p.clients[ci];
  const float* __restrict__ U = Ubase + (int64_t)ci * u_stride;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lg = lane >> 4;
  const int arow0 = b * kSRows + w * 32;
  const int ns = p.NS;

  float ub[2][NSMAX];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int row = arow0 + 16 * rt + li;
#pragma unroll
    for (int s = 0; s < NSMAX; ++s)
      ub[rt][s] = (s < ns) ? U[(int64_t)(lg * ns + s) * p.MP + row] : 0.f;
  }
  f4 accp[2][RT];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct) accp[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};

  double sl2 = 0.0, sl1 = 0.0, snz = 0.0;
  const float lam = p.lam;
  float* __restrict__ Sblk = p.S + cl.s_off;
  const float* __restrict__ Mb = cl.M;

  for (int j0 = 0; j0 < cl.n; j0 += 16) {
    const int vr = cl.vrow0 + j0;
    float va[NSMAX];
#pragma unroll
    for (int s = 0; s < NSMAX; ++s)
      va[s] = (s < ns) ? p.Vrow[(int64_t)(vr + li) * RP + lg * ns + s] : 0.f;
    f4 vb[RT];
#pragma unroll
    for (int ct = 0; ct < RT; ++ct)
      vb[ct] = *reinterpret_cast<const f4*>(p.Vcol + (int64_t)(16 * ct + li) * p.NVP + vr + 4 * lg);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int row = arow0 + 16 * rt + li;
      const bool rok = row < p.m;
      float mv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = j0 + 4 * lg + v;
        mv[v] = (rok && col < cl.n) ? Mb[(int64_t)col * cl.ldm + row] : 0.f;
      }
      f4 a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NSMAX; ++s)
        if (s < ns) a1 = mfma4(va[s], ub[rt][s], a1);
      f4 lamv;
      float l2 = 0.f, l1 = 0.f, nz = 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = j0 + 4 * lg + v;
        const float R = mv[v] - a1[v];
        const float L = fminf(fmaxf(R, -lam), lam);
        const float Sv = R - L;
        if (rok && col < cl.n) Sblk[(int64_t)col * p.lds + row] = Sv;
        lamv[v] = L;
        l2 += L * L;
        l1 += fabsf(Sv);
        nz += (Sv != 0.f) ? 1.f : 0.f;
      }
      sl2 += (double)l2;
      sl1 += (double)l1;
      snz += (double)nz;
#pragma unroll
      for (int ct = 0; ct < RT; ++ct)
#pragma unroll
        for (int s = 0; s < 4; ++s) accp[rt][ct] = mfma4(lamv[s], vb[ct][s], accp[rt][ct]);
    }
  }

  float* Pi = p.P + (int64_t)ci * RP * p.MP;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < RT; ++ct)
      *reinterpret_cast<f4*>(Pi + (int64_t)(16 * ct + li) * p.MP + arow0 + 16 * rt + 4 * lg) =
          accp[rt][ct];

  __shared__ double sred[4][3];
  sl2 = wave_sum(sl2);
  sl1 = wave_sum(sl1);
  snz = wave_sum(snz);
  if (lane == 0) {
    sred[w][0] = sl2;
    sred[w][1] = sl1;
    sred[w][2] = snz;
  }
  __syncthreads();
  if (tid == 0) {
    double* o = p.spart + ((int64_t)ci * p.nrb + b) * 4;
    o[0] = sred[0][0] + sred[1][0] + sred[2][0] + sred[3][0];
    o[1] = sred[0][1] + sred[1][1] + sred[2][1] + sred[3][1];
    o[2] = sred[0][2] + sred[1][2] + sred[2][2] + sred[3][2];
    o[3] = 0.0;
  }
}

// Partial Gram of 32 rows of a column-major U block (values in LDS as FP64).
__device__ void gram_rows_partial(const double (*ul)[kMaxRank + 1], int RP, double* out) {
  for (int e = threadIdx.x; e < RP * RP; e += blockDim.x) {
    const int a = e / RP, b = e % RP;
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < kURows; ++j) s += ul[j][a] * ul[j][b];
    out[e] = s;
  }
}

// ---------------------------------------------------------------------------
// U update. grid = (row blocks of 32, final ? 1 : E). Thread (a = tid % 32,
// cq = tid / 32) owns row a and rank columns cq, cq + 8, ...
// final = 1: U^(t+1) = mean_i U_i^new (eq. "U_agg") into the consensus buffer,
//            plus ||U^(t+1) - U^(t)||^2 partials; Gram slot 0.
// final = 0: per-client U_i^new (K > 1 intermediate local steps); Gram slot i.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_uupdate(DevParams p, const float* __restrict__ Uin,
                                                 int64_t uin_stride, float* __restrict__ Uout,
                                                 int64_t uout_stride,
                                                 const float* __restrict__ Uprev, int final_step,
                                                 double eta) {
  __shared__ double ul[kURows][kMaxRank + 1];
  __shared__ double dred[4];
  const int RP = p.RP, r = p.r, MP = p.MP;
  const int tid = threadIdx.x, al = tid & 31, cq = tid >> 5;
  const int a = blockIdx.x * kURows + al;
  const int nq = RP / 8;
  const int i_first = final_step ? 0 : (int)blockIdx.y;
  const int i_last = final_step ? p.E : (int)blockIdx.y + 1;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;

  for (int i = i_first; i < i_last; ++i) {
    const float* __restrict__ Ui = Uin + (int64_t)i * uin_stride;
    const float* __restrict__ Pi = p.P + (int64_t)i * RP * MP;
    const double ci = p.clients[i].c;
    if (p.u_mode == 0) {  // gradient step
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q < nq) {
          const int c = cq + 8 * q;
          const double u = Ui[(int64_t)c * MP + a];
          const double pv = Pi[(int64_t)c * MP + a];
          acc[q] += u - eta * (ci * u - pv);
        }
      }
    } else {  // closed form: P_i A_i + U_i B_i
      const double* __restrict__ Af = p.Afac + (int64_t)i * RP * RP;
      const double* __restrict__ Bf = p.Bfac + (int64_t)i * RP * RP;
      for (int k = 0; k < r; ++k) {
        const double pk = Pi[(int64_t)k * MP + a];
        const double uk = Ui[(int64_t)k * MP + a];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (q < nq) {
            const int c = cq + 8 * q;
            acc[q] += pk * Af[k * RP + c] + uk * Bf[k * RP + c];
          }
        }
      }
    }
  }
  const double scale = final_step ? 1.0 / (double)p.E : 1.0;
  float* __restrict__ Uo = Uout + (final_step ? 0 : (int64_t)blockIdx.y * uout_stride);
  double dsq = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (q < nq) {
      const int c = cq + 8 * q;
      const float v = (a < p.m && c < r) ? (float)(acc[q] * scale) : 0.f;
      Uo[(int64_t)c * MP + a] = v;
      ul[al][c] = (double)v;
      if (final_step) {
        const double d = (double)v - (double)Uprev[(int64_t)c * MP + a];
        dsq += d * d;
      }
    }
  }
  dsq = wave_sum(dsq);
  if ((tid & 63) == 0) dred[tid >> 6] = dsq;
  __syncthreads();
  const int slot = final_step ? 0 : (int)blockIdx.y;
  gram_rows_partial(ul, RP, p.gram_part + ((int64_t)slot * p.nub + blockIdx.x) * RP * RP);
  if (final_step && tid == 0) p.upart[blockIdx.x] = dred[0] + dred[1] + dred[2] + dred[3];
}

// Gram partials of the consensus U (start of the run).
__global__ __launch_bounds__(256) void k_gram_init(DevParams p, const float* __restrict__ U) {
  __shared__ double ul[kURows][kMaxRank + 1];
  const int RP = p.RP;
  for (int e = threadIdx.x; e < kURows * RP; e += blockDim.x) {
    const int al = e % kURows, c = e / kURows;
    ul[al][c] = (double)U[(int64_t)c * p.MP + blockIdx.x * kURows + al];
  }
  __syncthreads();
  gram_rows_partial(ul, RP, p.gram_part + (int64_t)blockIdx.x * RP * RP);
}

// ---------------------------------------------------------------------------
// Finalize: G = U^T U + rho I from the Gram partials, G^{-1} via FP64
// Cholesky, and (record = 1) the round statistics. grid = per_client ? E : 1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(DevParams p, double* Ginv, int64_t g_stride,
                                                  int per_client, int record) {
  __shared__ double A[kMaxRank * kMaxRank], X[kMaxRank * kMaxRank];
  const int r = p.r, RP = p.RP;
  __shared__ double tr_sh;
  __shared__ double red[8][4];
  const int tid = threadIdx.x;
  const int gi = blockIdx.x;
  const double* gp = p.gram_part + (int64_t)gi * p.nub * RP * RP;
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int a = e / r, b = e % r;
    double s = 0.0;
    for (int k = 0; k < p.nub; ++k) s += gp[(int64_t)k * RP * RP + a * RP + b];
    A[e] = s;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < r; ++k) t += A[k * r + k];
    tr_sh = t;
  }
  __syncthreads();
  for (int k = tid; k < r; k += blockDim.x) A[k * r + k] += p.rho;
  __syncthreads();
  spd_inverse(A, X, r, r);
  double* Gout = Ginv + (int64_t)gi * g_stride;
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    const int a = e / RP, b = e % RP;
    Gout[e] = (a < r && b < r) ? A[a * r + b] : 0.0;
  }
  if (per_client) {
    if (tid == 0) p.ucl_sq[gi] = tr_sh;
    return;
  }
  if (!record) {
    if (tid == 0) p.dstate->u_sq = tr_sh;
    return;
  }
  // Round statistics (FP64, fixed summation order).
  double l2 = 0.0, l1 = 0.0, nz = 0.0, vsq = 0.0, du = 0.0;
  const int nsp = p.E * p.nrb;
  for (int k = tid; k < nsp; k += blockDim.x) {
    l2 += p.spart[(int64_t)k * 4 + 0];
    l1 += p.spart[(int64_t)k * 4 + 1];
    nz += p.spart[(int64_t)k * 4 + 2];
  }
  for (int k = tid; k < p.ngroups * r; k += blockDim.x) {
    const int g = k / r, d = k % r;
    vsq += p.gv_part[(int64_t)g * RP * RP + d * RP + d];
  }
  for (int k = tid; k < p.nub; k += blockDim.x) du += p.upart[k];
  l2 = wave_sum(l2);
  l1 = wave_sum(l1);
  nz = wave_sum(nz);
  vsq = wave_sum(vsq);
  du = wave_sum(du);
  const int w = tid >> 6;
  if ((tid & 63) == 0) {
    red[w][0] = l2;
    red[w][1] = l1;
    red[w][2] = nz;
    red[w][3] = vsq;
    red[w + 4][0] = du;
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = blockDim.x >> 6;
    double s[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < nw; ++k) {
      s[0] += red[k][0];
      s[1] += red[k][1];
      s[2] += red[k][2];
      s[3] += red[k][3];
      s[4] += red[k + 4][0];
    }
    double ureg;
    if (p.K == 1) {
      ureg = 0.5 * p.rho * p.dstate->u_sq;
    } else {
      ureg = 0.0;
      for (int i = 0; i < p.E; ++i) ureg += 0.5 * p.clients[i].c * p.ucl_sq[i];
    }
    const int64_t t = p.dstate->t;
    StatsRec rec;
    rec.t = (double)t;
    rec.objective = 0.5 * s[0] + 0.5 * p.rho * s[3] + (double)p.lam * s[1] + ureg;
    rec.lambda_fro_sq = s[0];
    rec.nnz = s[2];
    rec.du_sq = s[4];
    rec.u_sq = tr_sh;
    rec.v_sq = s[3];
    rec.l1 = s[1];
    p.hist[t % kHist] = rec;
    p.dstate->t = t + 1;
    p.dstate->u_sq = tr_sh;
  }
}

// U^(0) into the padded column-major layout (zeros outside m x r).
__global__ void k_copy_in_U(DevParams p, const float* __restrict__ U0, int64_t ldu,
                            float* __restrict__ Ucol) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)p.RP * p.MP) return;
  const int a = (int)(e % p.MP), c = (int)(e / p.MP);
  Ucol[e] = (a < p.m && c < p.r) ? U0[(int64_t)c * ldu + a] : 0.f;
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
             (double)p.Vrow[(int64_t)(cl.vrow0 + j) * p.RP + c];
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
  V[(int64_t)c * ldv + col0 + j] = p.Vrow[(int64_t)(cl.vrow0 + j) * p.RP + c];
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
  const int span = (cl.n + kVCols - 1) / kVCols * kVCols;
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
hipError_t launch_vpass(const DevParams& p, const float* U, int64_t u_stride, const double* Ginv,
                        int64_t g_stride, hipStream_t st) {
  dim3 grid(p.ngroups), block(512);
  switch (p.RP / 16) {
    case 1: hipLaunchKernelGGL(k_vpass<1>, grid, block, 0, st, p, U, u_stride, Ginv, g_stride); break;
    case 2: hipLaunchKernelGGL(k_vpass<2>, grid, block, 0, st, p, U, u_stride, Ginv, g_stride); break;
    case 3: hipLaunchKernelGGL(k_vpass<3>, grid, block, 0, st, p, U, u_stride, Ginv, g_stride); break;
    case 4: hipLaunchKernelGGL(k_vpass<4>, grid, block, 0, st, p, U, u_stride, Ginv, g_stride); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_client_factor(const DevParams& p, hipStream_t st) {
  hipLaunchKernelGGL(k_client_factor, dim3(p.E), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_spass(const DevParams& p, const float* U, int64_t u_stride, hipStream_t st) {
  dim3 grid(p.nrb, p.E), block(256);
  switch (p.RP / 16) {
    case 1: hipLaunchKernelGGL(k_spass<1>, grid, block, 0, st, p, U, u_stride); break;
    case 2: hipLaunchKernelGGL(k_spass<2>, grid, block, 0, st, p, U, u_stride); break;
    case 3: hipLaunchKernelGGL(k_spass<3>, grid, block, 0, st, p, U, u_stride); break;
    case 4: hipLaunchKernelGGL(k_spass<4>, grid, block, 0, st, p, U, u_stride); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_uupdate(const DevParams& p, const float* Uin, int64_t uin_stride, float* Uout,
                          int64_t uout_stride, const float* Uprev_cons, int final_step,
                          double eta, hipStream_t st) {
  dim3 grid(p.nub, final_step ? 1 : p.E), block(256);
  hipLaunchKernelGGL(k_uupdate, grid, block, 0, st, p, Uin, uin_stride, Uout, uout_stride,
                     Uprev_cons, final_step, eta);
  return hipGetLastError();
}

hipError_t launch_finalize(const DevParams& p, double* Ginv, int64_t g_stride, int per_client,
                           int record, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(per_client ? p.E : 1), dim3(256), 0, st, p, Ginv,
                     g_stride, per_client, record);
  return hipGetLastError();
}

hipError_t launch_gram_init(const DevParams& p, const float* U, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_init, dim3(p.nub), dim3(256), 0, st, p, U);
  return hipGetLastError();
}

hipError_t launch_copy_in_U(const DevParams& p, const float* U0, int64_t ldu, float* Ucol,
                            hipStream_t st) {
  const int64_t tot = (int64_t)p.RP * p.MP;
  hipLaunchKernelGGL(k_copy_in_U, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p, U0,
                     ldu, Ucol);
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
    const int span = (host_clients[i].n + kVCols - 1) / kVCols * kVCols;
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

}  // namespace rpca
