// Internal definitions shared by the DCF-PCA kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rpca {

constexpr int kMaxRank = 128;    // largest supported factor rank r
// Ranks up to kFoldMaxRP (four 16-rank tiles) take every launch shape, the
// BF16 passes, and the finalize folded into the V-pass; wider ones (five to
// eight rank tiles) run the FP32 passes with one column group per V-pass wave
// and one S-pass column phase, full rank tiles (NS = RP / 4), and a
// standalone finalize.
constexpr int kFoldMaxRP = 64;
constexpr int kHist = 4096;      // per-round statistics kept in a ring
constexpr int kVCols = 32;       // columns per V-finalize work-group
constexpr int kVPad = 64;        // client V blocks are padded to multiples of 64 rows
constexpr int kVStreamCols = 64; // columns per V-pass streaming work-group (4 waves x 16)
constexpr int kSRows = 128;      // rows per S-pass work-group (4 waves x 32 rows)
constexpr int kURows = 64;       // rows per U-update work-group

// Factor storage. A factor X (U: MP rows, V: NVP rows; RP = r rounded up to 16
// ranks, zero padded) is kept in three layouts in one block of floats:
//   col : column-major, leading dimension = rows            (RP * rows)
//   pa  : MFMA A-operand packing, for 16-row chunk ch, step s < NS, lane l:
//         X[16 ch + l % 16][(l / 16) * NS + s]                (4 * NS * rows)
//   pb  : MFMA B-operand packing, for chunk ch, rank tile ct, lane l, e < 4:
//         X[16 ch + 4 (l / 16) + e][16 ct + l % 16]           (RP * rows)
// so that every operand a wave needs for one 16x16x4 MFMA step is a single
// contiguous 256 B (pa) or 1 KiB (pb) read. V additionally keeps a row-major
// copy (rows x RP) in front of its factor block.
// When the last rank tile holds at most 12 ranks, products whose output
// dimension is the rank use 4x4 MFMA blocks for it, one per group of four
// ranks ("quads"), instead of a zero-padded 16x16 tile:
//   nquads = ceil(r/4) - 4 (RP/16 - 1) if that is <= 3, else 0,
// and the factor keeps a fourth layout for them:
//   pq  : for chunk ch, quad q, g < 4, j < 4, e < 4 (16 floats per (ch, q, g)):
//         X[16 ch + 4 g + e][RP - 16 + 4 q + j]               (4 * nquads * rows)
__host__ __device__ constexpr int nquads(int RP, int NS) {
  return NS - 4 * (RP / 16 - 1) <= 3 ? NS - 4 * (RP / 16 - 1) : 0;
}
__host__ __device__ inline int64_t fb_floats(int64_t rows, int RP, int NS) {
  return 2 * (int64_t)RP * rows + 4 * (int64_t)NS * rows + 4 * (int64_t)nquads(RP, NS) * rows;
}
__host__ __device__ inline int64_t fb_pa_off(int64_t rows, int RP) { return (int64_t)RP * rows; }
__host__ __device__ inline int64_t fb_pb_off(int64_t rows, int RP, int NS) {
  return (int64_t)RP * rows + 4 * (int64_t)NS * rows;
}
__host__ __device__ inline int64_t fb_pq_off(int64_t rows, int RP, int NS) {
  return 2 * (int64_t)RP * rows + 4 * (int64_t)NS * rows;
}
// V buffer: row-major NVP x RP copy, then the factor block.
__host__ __device__ inline int64_t vbuf_floats(int64_t NVP, int RP, int NS) {
  return (int64_t)NVP * RP + fb_floats(NVP, RP, NS);
}
__host__ __device__ inline float* v_fb(float* V, int64_t NVP, int RP) { return V + NVP * RP; }
__host__ __device__ inline const float* v_fb(const float* V, int64_t NVP, int RP) {
  return V + NVP * RP;
}

// BF16 operand packings (mixed-precision rounds, v_mfma_f32_16x16x32_bf16,
// whose lane l supplies A[l%16][8 (l/16) + e] and B[8 (l/16) + e][l%16],
// e < 8, and receives D[4 (l/16) + v][l%16]). RK = 32 ceil(r/32) ranks on the
// contraction side (NK = RK / 32 blocks), RP ranks on the output side; rows is
// a multiple of 32 and every entry past the factor's rows or rank is 0.
// Element (a, c) of a factor X lives in
//   hA : 16-row chunk ch, block kb: X[16 ch + l%16][32 kb + 8 (l/16) + e]
//   hP : 32-row chunk ch, half t, block kb:
//        X[32 ch + 8 ((l%16)/4) + 4 t + l%4][32 kb + 8 (l/16) + e]
//        (rows permuted so that a product with this operand on the A side
//        leaves lane l the rows 8 (l/16) + 4 t + v, i.e. with both halves the
//        eight consecutive rows 8 (l/16) + e)
//   hB : 32-row chunk ch, rank tile ct: X[32 ch + 8 (l/16) + e][16 ct + l%16]
// each as 64 lanes x 8 bf16 = 1 KiB per operand. Sizes in bf16 elements:
// hA and hP rows * RK, hB rows * RP, in that order. Two such blocks follow
// each other: hi = x rounded to BF16, then lo = (x - hi) rounded to BF16, so
// that hi + lo carries 16 significand bits (three-product rounds, X3).
__host__ __device__ inline int64_t hb_elems(int64_t rows, int RK, int RP) {
  return rows * (2 * (int64_t)RK + RP);
}
__host__ __device__ inline int64_t hb_hA(int a, int c, int NK) {
  return ((((int64_t)(a >> 4) * NK + (c >> 5)) * 64 + 16 * ((c & 31) >> 3) + (a & 15)) << 3) + (c & 7);
}
__host__ __device__ inline int64_t hb_hP(int a, int c, int NK) {
  const int w = a & 31, t = (w >> 2) & 1, i = 4 * (w >> 3) + (w & 3);
  return (((((int64_t)(a >> 5) * 2 + t) * NK + (c >> 5)) * 64 + 16 * ((c & 31) >> 3) + i) << 3) + (c & 7);
}
__host__ __device__ inline int64_t hb_hB(int a, int c, int RT) {
  return ((((int64_t)(a >> 5) * RT + (c >> 4)) * 64 + 16 * ((a & 31) >> 3) + (c & 15)) << 3) + (a & 7);
}
// BF16 copies of M, two layouts (client i's block starts at vrow0_i * MP
// elements and spans MP rows by NVc_i = n_i rounded up to 64 columns, zero
// padded):
//   V-pass layout, 16-column group cg, 32-row chunk ch:
//        M[32 ch + 8 (l/16) + e][16 cg + l%16]   at ((cg (MP/32) + ch) 64 + l) 8 + e
//   S-pass layout, 16-row tile rt, 32-column chunk cc:
//        M[16 rt + l%16][32 cc + 8 (l/16) + e]   at ((rt (NVc/32) + cc) 64 + l) 8 + e

// Sparse S (RPCA_FLAG_SPARSE_S). The S-pass writes S in tiles of 16 rows by
// 16 columns of the padded V rows: tile = (column / 16) * (MP / 16) + row / 16.
// A tile has 64 slots of four entries, slot b = 16 a + 4 g + v holding rows
// 4 g + e (e < 4) of column 4 a + v (the four rows one V-pass lane reads
// together), one 64-bit slot word (bit b set: slot b has a nonzero entry),
// and room for 64 slots of values (256 floats), of which the nonzero slots
// fill the front, as float4, in slot order.
constexpr int kSparseVals = 256;
__host__ __device__ inline int64_t sparse_tile(int MP, int64_t vcol, int row) {
  return (vcol >> 4) * (int64_t)(MP >> 4) + (row >> 4);
}
// What of S an S-pass tile writes besides its statistics and U-step term.
enum SOutMode { kSOutNone = 0, kSOutDense = 1, kSOutSparse = 2 };

// One client (Section 2.1): its borrowed block M_i and where its private
// state lives in the workspace.
struct ClientDev {
  const float* M;   // column-major m x n_i, leading dimension ldm
  int64_t ldm;
  int64_t s_off;    // first float of S_i in the S buffer (leading dimension lds)
  int64_t col0;     // first global column of the client
  int32_t n;        // n_i
  int32_t vrow0;    // first row of V_i in the padded V buffers (multiple of 64)
  int32_t g0, g1;   // V-finalize work-groups [g0, g1) that cover this client
  double c;         // rho * n_i / n
  int32_t idx;      // client index i
  int32_t pad;
};

// A V-pass work unit: up to 32 (finalize) or 64 (streaming) consecutive
// columns of one client.
struct VGroup {
  int32_t client, j0, ncols, vrow;  // vrow: first row in the padded V buffers
};

// A V-pass streaming work unit (up to 64 columns of one client) with its
// client's record inline, so that a work-group needs one table read.
struct VTile {
  ClientDev cl;
  int32_t client, j0, ncols, pad;
};

// Device-resident scalars carried from round to round.
struct DevState {
  int64_t t;                 // rounds finished
  double u_sq;               // ||U^(t)||_F^2 (trace of the current Gram)
  double u_sq_next;          // trace of the new Gram until the round is recorded
  double pad[5];
};

struct StatsRec {  // mirrors rpca_stats
  double t, objective, lambda_fro_sq, nnz, du_sq, u_sq, v_sq, l1, objective_target;
};

struct DevParams {
  int32_t m, MP, r, RP, NS, E, K;
  int32_t NVP;           // padded rows of the V buffers
  int64_t n;             // total columns
  int64_t lds;           // leading dimension of S (= m rounded up to 4)
  int64_t ublock;        // floats of one U factor block, fb_floats(MP, RP, NS)
  int32_t nrb;           // S-pass row blocks (MP / kSRows)
  int32_t nub;           // U-update row blocks (MP / kURows)
  int32_t ngroups;       // V-finalize work-groups (32 columns each)
  int32_t ng64;          // V-pass streaming column groups (64 columns each)
  int32_t vsplit;        // V-pass row splits
  int32_t vsplit_rows;   // rows per V-pass row split (multiple of 16)
  int32_t vcols;         // 16-column groups per FP32 V-pass wave (1 or 4)
  int32_t sphases;       // column phases of the FP32 S-pass work-groups (1: 256, 2: 512 threads)
  int32_t vqueue;        // 1: V-pass as a persistent launch over a tile queue
  int32_t squeue;        // 1: S-pass as a persistent launch over a tile queue
  uint32_t* queue;       // tile-queue counters: [0, 1] V-pass, [2, 3] S-pass (zero between launches)
  int32_t u_mode, eta_sched;
  float lam;             // lambda of the rounds being enqueued
  float lam_rec;         // lambda of the last enqueued round (its deferred record)
  float lam_target;      // lambda of the problem (rpca_params), the schedule's target
  int32_t huber;         // 1: the S-pass sums H_{lam_target}(R) (lam != lam_target)
  double omega;          // multiplier of the consensus U step (1: the method's step)
  double rho, eta0;
  const ClientDev* clients;
  const ClientDev* clients_lpt;  // the same records, widest client first (S-pass order)
  const VGroup* vgroups;
  const VTile* vg64;
  float* S;              // all clients' S_i (stored-S layout only)
  float* V;              // V buffer this launch writes or reads (see vbuf_floats)
  float* Wpart;          // V-pass partial W per row split, [vsplit][NVP][RP]
  float* P;              // per-client U-step term T_i, column-major MP x RP
  double* gv_part;       // per V-finalize group partial V^T V, RP x RP
  double* gv_tr;         // per V-finalize group trace of its partial V^T V
  double* Afac;          // per-client (V_i^T V_i + c_i I)^{-1}, RP x RP
  double* gram_part;     // per (client,) U row block partial U^T U, RP x RP
  double* spart;         // per S-pass work-group: sums of Lambda^2, |S|, nnz(S)
  double* upart;         // per U row block: ||dU||^2
  double* ucl_sq;        // per-client ||U_i||^2 of the current local factors
  DevState* dstate;
  StatsRec* hist;
  double* stat_part;     // seven round statistics (finalize folded into the V-pass)
  // Mixed precision (RPCA_FLAG_BF16): factor blocks carry the BF16 packings
  // after their FP32 layouts (U: at ublock floats; V: at vbuf_floats), and M
  // has two BF16 copies.
  int32_t bf16;          // 1: keep the BF16 packings (hi and lo) up to date
  int32_t RK, NK;        // contraction-side ranks (32 NK) and blocks
  uint16_t* Mbv;         // BF16 M, V-pass layout
  uint16_t* Mbs;         // BF16 M, S-pass layout
  // Sparse S (RPCA_FLAG_SPARSE_S): support words and values of every piece.
  uint64_t* Smask;
  float* Sval;
};

// BF16 packings of a U factor block / a V buffer.
__host__ __device__ inline uint16_t* u_hb(float* U, const DevParams& p) {
  return reinterpret_cast<uint16_t*>(U + p.ublock);
}
__host__ __device__ inline const uint16_t* u_hb(const float* U, const DevParams& p) {
  return reinterpret_cast<const uint16_t*>(U + p.ublock);
}
__host__ __device__ inline uint16_t* v_hb(float* V, const DevParams& p) {
  return reinterpret_cast<uint16_t*>(V + vbuf_floats(p.NVP, p.RP, p.NS));
}
__host__ __device__ inline const uint16_t* v_hb(const float* V, const DevParams& p) {
  return reinterpret_cast<const uint16_t*>(V + vbuf_floats(p.NVP, p.RP, p.NS));
}

// Launch helpers (kernels live in rpca_vpass.hip, rpca_spass.hip, rpca_bf16.hip
// and rpca_tail.hip).
// Factor distance: work-groups per side (64 at widths up to 64, 16 at 128),
// Gram entries per work-group, and the doubles of its two workspaces (the
// same at both widths).
constexpr int dist_blocks(int W) { return W <= 64 ? 64 : 16; }
constexpr int kDistSlice = 3 * 64 * 64;
constexpr int64_t kDistPartDoubles = 2 * 64 * (int64_t)kDistSlice;
constexpr int kDistPart2Doubles = 3 * kMaxRank * kMaxRank / 256;
// S source for the V-pass: zero, the stored S buffer, recomputed from the
// previous round's factors, or the sparse S the previous S-pass wrote.
enum VMode { kSZero = 0, kSStored = 1, kSRecompute = 2, kSSparse = 3 };
// V-pass, streaming part: partial W = (M_i - S_i)^T U_i per row split into
// p.Wpart. U: factor block of the input U (client stride u_stride); Uold /
// Vold: previous U factor block and previous V buffer (kSRecompute).
// fin_Ginv != NULL: two extra work-groups run the previous round's finalize
// (Gram inverse into fin_Ginv; statistics) alongside the streaming ones.
hipError_t launch_vpass(const DevParams& p, int mode, const float* U, int64_t u_stride,
                        const float* Uold, const float* Vold, double* fin_Ginv, hipStream_t st);
// V-pass, finishing part: V = W G^{-1} into p.V, and the V_i^T V_i partials;
// rec = 1 also records the previous round (its finalize ran in the V-pass).
hipError_t launch_vfinal(const DevParams& p, const double* Ginv, int64_t g_stride, int rec,
                         hipStream_t st);
hipError_t launch_client_factor(const DevParams& p, hipStream_t st);
// S-pass over clients [client_base, client_base + client_count) with V = p.V.
// Sout/lds_out: column-major buffer S is written to, indexed by global column
// (NULL: S is not stored); emit_only: write S only (no U-step term, no
// statistics).
hipError_t launch_spass(const DevParams& p, const float* U, int64_t u_stride, float* Sout,
                        int64_t lds_out, int emit_only, int client_base, int client_count,
                        hipStream_t st);
// U update into factor block(s) Uout; Uprev_col: column-major previous U.
hipError_t launch_uupdate(const DevParams& p, float* Uout, int64_t uout_stride,
                          const float* Uprev_col, int final_step, hipStream_t st);
hipError_t launch_finalize(const DevParams& p, double* Ginv, int64_t g_stride, int per_client,
                           int record, hipStream_t st);
hipError_t launch_gram_init(const DevParams& p, const float* Ucol, hipStream_t st);
hipError_t launch_copy_in_U(const DevParams& p, const float* U0, int64_t ldu, float* Ufb,
                            hipStream_t st);
// U^(0) with i.i.d. N(0, 1) entries drawn from `seed` (SplitMix64 counters and
// Box-Muller; the rule is stated with rpca_init) into a factor block.
hipError_t launch_init_U_gauss(const DevParams& p, uint64_t seed, float* Ufb, hipStream_t st);
hipError_t launch_materialize(const DevParams& p, const ClientDev* host_clients,
                              const int64_t* col_off, const float* Ucol, int client_begin,
                              int client_end, float* L, int64_t ldl, float* S, int64_t lds,
                              hipStream_t st);
hipError_t launch_get_factors(const DevParams& p, const ClientDev* host_clients,
                              const int64_t* col_off, const float* Ucol, float* U, int64_t ldu,
                              float* V, int64_t ldv, hipStream_t st);
hipError_t launch_pack_target(const DevParams& p, const ClientDev* host_clients,
                              const int64_t* col_off, const float* Us, int64_t ldus,
                              const float* Vs, int64_t ldvs, int rs, float* Ut, float* Vt,
                              int RPT, hipStream_t st);
// ||X1 Y1^T - X2 Y2^T||_F^2 -> out2[0] and ||X2 Y2^T||_F^2 -> out2[1], from
// Gram matrices (FP64). X*: column-major, MP rows (ld MP); Y*: column-major,
// NVP rows (ld NVP); widths rp1, rp2 <= kMaxRank. part: kDistPartDoubles
// doubles; part2: kDistPart2Doubles doubles.
// Mixed precision (rpca_bf16.hip). The BF16 copies of M from the borrowed
// FP32 blocks (zero padded).
hipError_t launch_m_to_bf16(const DevParams& p, hipStream_t st);
// BF16 V-pass (streaming part) and S-pass; same outputs and work-group roles
// as launch_vpass (mode kSZero or kSRecompute) and launch_spass (all clients,
// no S output).
// x3 = 1: M read in FP32 from the caller's blocks and every product formed
// from hi/lo splits (three BF16 products).
hipError_t launch_vpass_h(const DevParams& p, int mode, const float* U, const float* Uold,
                          const float* Vold, double* fin_Ginv, int x3, hipStream_t st);
hipError_t launch_spass_h(const DevParams& p, const float* U, int x3, hipStream_t st);

hipError_t launch_factor_distance(const DevParams& p, const float* X1, const float* Y1, int rp1,
                                  const float* X2, const float* Y2, int rp2, double* part,
                                  double* part2, double* out2, hipStream_t st);

}  // namespace rpca
