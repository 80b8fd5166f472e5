// C ABI of the DCF-PCA library: argument checks, workspace carving, the
// per-round launch sequence of Algorithm 1 (Section 2.2) and the solve loop.
#include "../../include/rpca.h"
#include "rpca_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace rpca;

struct rpca_ctx {
  DevParams p{};
  std::vector<ClientDev> clients;
  std::vector<ClientDev> clients_lpt;  // widest first
  std::vector<VGroup> vgroups;
  std::vector<int64_t> col_off;  // first global column of each client, [E + 1]
  hipStream_t stream = nullptr;
  int64_t rounds = 0;
  // The last local step's finalize (Gram inverse of the new U and the round
  // statistics) is deferred into the next round's V-pass launch, which runs it
  // in one extra work-group next to the streaming ones. Calls that read its
  // outputs flush it first with a standalone launch.
  bool fin_pending = false;
  // RPCA_FLAG_GRAPH: two-round graphs, one per starting buffer parity.
  bool use_graph = false;
  int32_t vsplit_max = 1;  // largest V-pass row-split count the workspace holds
  int32_t prec = RPCA_PREC_FP32;  // precision of the streaming passes
  int64_t max_ldm = 0;            // largest leading dimension of the M blocks
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int cur = 0;   // consensus U buffer holding U^(t)
  int vcur = 0;  // V buffer holding the latest V
  int inner = 1;
  bool recompute = false;  // S rebuilt from (U_prev, V) instead of stored
  // RPCA_FLAG_SPARSE_S: the sparse S in the workspace is that of the last
  // round's S-pass (an FP32 round); lam_rec is its lambda.
  bool sparse_valid = false;
  // With RPCA_FLAG_SPARSE_S: 1 while the launch shape hands S over in sparse
  // form, 0 while FP32 rounds rebuild it (the autotuner decides).
  int32_t use_sparse = 0;
  float* V[2] = {nullptr, nullptr};  // V buffers (row-major copy + factor block)
  std::vector<VTile> vg64;
  bool poisoned = false;
  std::string err;
  float* U[2] = {nullptr, nullptr};
  float* Uc[2] = {nullptr, nullptr};
  double* Ginv = nullptr;  // slot 0: consensus; slots 1..E: per-client (K > 1)
  float* Uprev = nullptr;
  float* Vprev = nullptr;
  bool have_prev = false;
  float* Ut = nullptr;
  float* Vt = nullptr;
  int RPT = 0;
  bool have_target = false;
  double* dpart = nullptr;
  double* dpart2 = nullptr;
  double* dout = nullptr;
  // The workspace, and the byte ranges in it that belong to this context
  // only (client tables holding its M pointers, the BF16 copies of its M);
  // rpca_copy_state copies everything else.
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<std::pair<size_t, size_t>> own_ranges;
  std::vector<int64_t> widths;
  int static_dev = -1;  // GPU whose static workspace this context uses (rpca_init_static)
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct Layout {
  size_t S, Smask, Sval, U0, U1, Uc0, Uc1, V0, V1, Mbv, Mbs, Wpart, P, gv, gvtr, Af, gram, spart, upart,
      ucl, Ginv, dstate, hist, stat_part, clients, clients_lpt, vgroups, vg64, Uprev, Vprev, Ut, Vt, dpart, dpart2, dout,
      queue, total;
  int32_t MP, RP, NS, NVP, nrb, nub, ngroups, ng64, vsplit, vsplit_rows, vsplit_max, RK;
  bool recompute, bf16, mcopy;
  int64_t lds, n, Sfloats;
};

const char* check_params(const rpca_params* p) {
  if (!p) return "params is NULL";
  if (p->m < 1 || p->m >= (int64_t)1 << 26) return "m must be in [1, 2^26)";
  if (p->E < 1 || p->E > 4096) return "E must be in [1, 4096]";
  if (!p->n_cols) return "n_cols is NULL";
  int64_t n = 0;
  for (int i = 0; i < p->E; ++i) {
    if (p->n_cols[i] < 1 || p->n_cols[i] > (int64_t)1 << 30) return "every n_i must be in [1, 2^30]";
    n += p->n_cols[i];
  }
  if (n > (int64_t)1 << 31) return "total columns n must be <= 2^31";
  if (p->r < 1 || p->r > kMaxRank) return "r must be in [1, 128]";
  {
    // The kernels address whole factor layouts through buffer resources with
    // 32-bit byte ranges: (m rounded up to 128) x (r rounded up to 16) and
    // (the clients' widths each rounded up to 64, summed) x (r rounded up to
    // 16) floats must each span fewer than 2^31 bytes.
    const int64_t RP = round_up(p->r, 16);
    int64_t nvp = 0;
    for (int i = 0; i < p->E; ++i) nvp += round_up(p->n_cols[i], kVPad);
    if (round_up(p->m, kSRows) * RP * 4 >= ((int64_t)1 << 31))
      return "m rounded up to 128, times r rounded up to 16, times 4 bytes must be < 2^31";
    if (nvp * RP * 4 >= ((int64_t)1 << 31))
      return "the sum of the n_i rounded up to 64, times r rounded up to 16, times 4 bytes must "
             "be < 2^31";
  }
  if (!(p->rho > 0.0) || !std::isfinite(p->rho)) return "rho must be finite and > 0";
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return "lambda must be finite and >= 0";
  if (p->K < 1 || p->K > 1024) return "K must be in [1, 1024]";
  if (p->inner < 1 || p->inner > 1024) return "inner must be in [1, 1024]";
  if (p->u_mode != RPCA_U_GRAD && p->u_mode != RPCA_U_CLOSED) return "unknown u_mode";
  if (p->u_mode == RPCA_U_GRAD && (!(p->eta0 > 0.0) || !std::isfinite(p->eta0)))
    return "eta0 must be finite and > 0 for RPCA_U_GRAD";
  if (p->eta_sched != RPCA_ETA_CONST && p->eta_sched != RPCA_ETA_SQRT) return "unknown eta_sched";
  if (p->flags & ~(uint32_t)(RPCA_FLAG_STORE_S | RPCA_FLAG_GRAPH | RPCA_FLAG_BF16 |
                             RPCA_FLAG_BF16X3 | RPCA_FLAG_SPARSE_S))
    return "unknown flags";
  if ((p->flags & RPCA_FLAG_SPARSE_S) &&
      (p->K != 1 || p->inner != 1 || (p->flags & RPCA_FLAG_STORE_S)))
    return "RPCA_FLAG_SPARSE_S needs K = 1, inner = 1 and no RPCA_FLAG_STORE_S";
  if ((p->flags & (RPCA_FLAG_BF16 | RPCA_FLAG_BF16X3)) &&
      (p->K != 1 || p->inner != 1 || (p->flags & RPCA_FLAG_STORE_S)))
    return "RPCA_FLAG_BF16 and RPCA_FLAG_BF16X3 need K = 1, inner = 1 and no RPCA_FLAG_STORE_S";
  if ((p->flags & (RPCA_FLAG_BF16 | RPCA_FLAG_BF16X3)) && p->r > kFoldMaxRP)
    return "RPCA_FLAG_BF16 and RPCA_FLAG_BF16X3 need r <= 64";
  return nullptr;
}

Layout make_layout(const rpca_params* p) {
  Layout L{};
  L.MP = (int32_t)round_up(p->m, kSRows);
  L.RP = (int32_t)round_up(p->r, 16);
  // Rank steps of the packed A operands: ceil(r/4) up to r = 64; beyond,
  // whole rank tiles (the padding ranks are zero).
  L.NS = L.RP <= kFoldMaxRP ? (p->r + 3) / 4 : L.RP / 4;
  L.lds = round_up(p->m, 4);
  L.RK = (int32_t)round_up(p->r, 32);
  L.bf16 = (p->flags & (RPCA_FLAG_BF16 | RPCA_FLAG_BF16X3)) != 0;
  L.mcopy = (p->flags & RPCA_FLAG_BF16) != 0;
  L.nrb = L.MP / kSRows;
  L.nub = L.MP / kURows;
  int64_t nvp = 0, ng = 0, ng64 = 0, n = 0;
  for (int i = 0; i < p->E; ++i) {
    nvp += round_up(p->n_cols[i], kVPad);
    ng += (p->n_cols[i] + kVCols - 1) / kVCols;
    ng64 += (p->n_cols[i] + kVStreamCols - 1) / kVStreamCols;
    n += p->n_cols[i];
  }
  L.NVP = (int32_t)nvp;
  L.ngroups = (int32_t)ng;
  L.ng64 = (int32_t)ng64;
  L.n = n;
  // Row splits of the V-pass: enough work-groups to fill the chip (>= 1024),
  // each covering at least 64 rows.
  {
    const int64_t want = (1024 + ng64 - 1) / ng64;
    const int64_t maxs = (p->m + 63) / 64;
    int64_t vs = want < maxs ? want : maxs;
    if (vs < 1) vs = 1;
    // BF16 rounds walk 32-row chunks.
    const int64_t rows = round_up((p->m + vs - 1) / vs, L.bf16 ? 32 : 16);
    L.vsplit_rows = (int32_t)rows;
    L.vsplit = (int32_t)((p->m + rows - 1) / rows);
    // rpca_autotune may try up to twice as many splits, and at least 8: the
    // work-group count decides how full the last wave of work-groups runs
    // (at m = 20000, n = 100000 the default is 1 split, and 2 give 6.1
    // waves of 512 resident work-groups).
    const int64_t vwant = 2 * L.vsplit > 8 ? 2 * L.vsplit : 8;
    const int64_t vmax = vwant < maxs ? vwant : maxs;
    L.vsplit_max = (int32_t)(vmax > L.vsplit ? vmax : L.vsplit);
  }
  L.recompute = p->K == 1 && p->inner == 1 && !(p->flags & RPCA_FLAG_STORE_S);
  L.Sfloats = L.recompute ? 0 : L.lds * n;
  const int E = p->E;
  const bool multi = p->K > 1;
  const size_t f = sizeof(float), d = sizeof(double);
  const size_t RR = (size_t)L.RP * L.RP;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.S = take((size_t)L.Sfloats * f);
  // Sparse S: per 16 x 16 tile of (row, padded column), a slot word and room
  // for 256 values.
  const bool sparse = (p->flags & RPCA_FLAG_SPARSE_S) != 0;
  const size_t tiles = sparse ? (size_t)(L.NVP / 16) * (size_t)(L.MP / 16) : 0;
  L.Smask = take(tiles * sizeof(uint64_t));
  L.Sval = take(tiles * kSparseVals * f);
  const size_t ub = (size_t)fb_floats(L.MP, L.RP, L.NS);
  // BF16 packings (hi, then lo) follow the FP32 layouts of each U block and V
  // buffer.
  const size_t uh = L.bf16 ? (size_t)hb_elems(L.MP, L.RK, L.RP) : 0;
  const size_t vh = L.bf16 ? (size_t)hb_elems(L.NVP, L.RK, L.RP) : 0;
  L.U0 = take((ub + uh) * f);
  L.U1 = take((ub + uh) * f);
  L.Uc0 = take(multi ? (size_t)E * ub * f : 0);
  L.Uc1 = take(multi ? (size_t)E * ub * f : 0);
  L.V0 = take(((size_t)vbuf_floats(L.NVP, L.RP, L.NS) + vh) * f);
  L.V1 = take(((size_t)vbuf_floats(L.NVP, L.RP, L.NS) + vh) * f);
  const size_t mh = L.mcopy ? (size_t)L.NVP * L.MP * sizeof(uint16_t) : 0;
  L.Mbv = take(mh);
  L.Mbs = take(mh);
  L.Wpart = take((size_t)(L.vsplit_max + 1) * L.NVP * L.RP * f);
  L.P = take((size_t)E * L.RP * L.MP * f);
  L.gv = take((size_t)L.ngroups * RR * d);
  L.gvtr = take((size_t)L.ngroups * d);
  L.Af = take((size_t)E * RR * d);
  L.gram = take((size_t)(multi ? E : 1) * L.nub * RR * d);
  L.spart = take((size_t)E * L.nrb * 4 * d);
  L.upart = take((size_t)L.nub * d);
  L.ucl = take((size_t)E * d);
  L.Ginv = take((size_t)(1 + (multi ? E : 0)) * RR * d);
  L.dstate = take(sizeof(DevState));
  L.hist = take((size_t)kHist * sizeof(StatsRec));
  L.stat_part = take((size_t)8 * d);
  L.clients = take((size_t)E * sizeof(ClientDev));
  L.clients_lpt = take((size_t)E * sizeof(ClientDev));
  L.vgroups = take((size_t)L.ngroups * sizeof(VGroup));
  L.vg64 = take((size_t)L.ng64 * sizeof(VTile));
  L.Uprev = take((size_t)L.RP * L.MP * f);
  L.Vprev = take((size_t)L.NVP * L.RP * f);
  L.Ut = take((size_t)kMaxRank * L.MP * f);
  L.Vt = take((size_t)L.NVP * kMaxRank * f);
  L.dpart = take((size_t)kDistPartDoubles * d);
  L.dpart2 = take((size_t)kDistPart2Doubles * d);
  L.dout = take((size_t)2 * d);
  L.queue = take(4 * sizeof(uint32_t));
  L.total = o;
  return L;
}

rpca_status fail(rpca_ctx* c, rpca_status st, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (st == RPCA_EDEVICE || st == RPCA_ENONFINITE) c->poisoned = true;
  }
  return st;
}

// Cause of the last failed context creation on this thread (rpca_last_error
// with no context).
thread_local std::string g_init_err;

rpca_status init_fail(rpca_status st, const std::string& msg) {
  g_init_err = msg;
  return st;
}

rpca_status dev_fail(rpca_ctx* c, hipError_t e, const char* where) {
  return fail(c, RPCA_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define RPCA_HIP(c, call, where)                 \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return dev_fail((c), e_, (where)); \
  } while (0)

// Optional per-kernel event timing (rpca_profile): a pair of events around
// every launch, grouped by phase.
struct Profiler {
  std::vector<hipEvent_t> ev;
  std::vector<int> phase;
  hipError_t begin(hipStream_t st, int ph) {
    hipEvent_t a;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    ev.push_back(a);
    phase.push_back(ph);
    return hipEventRecord(a, st);
  }
  hipError_t end(hipStream_t st) {
    hipEvent_t b;
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    ev.push_back(b);
    return hipEventRecord(b, st);
  }
  ~Profiler() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

#define RPCA_LAUNCH(c, prof, ph, call, where)                      \
  do {                                                              \
    if (prof) RPCA_HIP(c, (prof)->begin((c)->stream, (ph)), "event"); \
    RPCA_HIP(c, (call), (where));                                   \
    if (prof) RPCA_HIP(c, (prof)->end((c)->stream), "event");         \
  } while (0)

// Device parameters of a launch that reads or writes V buffer `v`.
DevParams with_v(const rpca_ctx* c, int v) {
  DevParams q = c->p;
  q.V = c->V[v];
  return q;
}

// Ranks above 64 fold no finalize into the V-pass (its r x r FP64 matrix
// would not share the V-pass LDS): a pending one runs as its own launch,
// recording the previous round, before the round's first V-pass.
hipError_t unfold_finalize(rpca_ctx* c, Profiler* prof) {
  if (!c->fin_pending || c->p.RP <= kFoldMaxRP) return hipSuccess;
  hipError_t e = prof ? prof->begin(c->stream, RPCA_PHASE_FINALIZE) : hipSuccess;
  if (e == hipSuccess) e = launch_finalize(c->p, c->Ginv, 0, 0, 1, c->stream);
  if (e == hipSuccess && prof) e = prof->end(c->stream);
  if (e == hipSuccess) c->fin_pending = false;
  return e;
}

// One round of Algorithm 1: K local steps (each: `inner` V/S alternations,
// then the U step) and the consensus mean at the last one.
rpca_status enqueue_round(rpca_ctx* c, Profiler* prof = nullptr) {
  // Rounds at another lambda than the problem's sum the Huber form of the
  // objective at the target lambda in their S-pass.
  c->p.huber = c->p.lam != c->p.lam_target ? 1 : 0;
  const DevParams& p = c->p;
  hipStream_t st = c->stream;
  const int64_t ustride = p.ublock;
  const int64_t gstride = (int64_t)p.RP * p.RP;
  const float* Ucons = c->U[c->cur];
  if (c->recompute) {
    // K = 1, one alternation: S of the previous round is rebuilt inside the
    // V-pass from (U^(t-1), V^(t)) and never stored.
    const bool h = c->prec != RPCA_PREC_FP32;
    // With RPCA_FLAG_SPARSE_S an FP32 round reads the S of the previous
    // round's S-pass when that was an FP32 round at this lambda.
    const bool sparse_in = !h && c->use_sparse && c->sparse_valid && p.lam == p.lam_rec;
    const int mode = c->rounds == 0 ? kSZero : sparse_in ? kSSparse : kSRecompute;
    const int vn = c->vcur ^ 1;
    DevParams q = with_v(c, vn);
    // BF16 rounds, and rounds whose launch shape rebuilds S, write no sparse S.
    if (h || !c->use_sparse) q.Smask = nullptr, q.Sval = nullptr;
    RPCA_HIP(c, unfold_finalize(c, prof), "finalize launch");
    double* fin = c->fin_pending ? c->Ginv : nullptr;
    c->fin_pending = false;
    const int x3 = c->prec == RPCA_PREC_BF16X3 ? 1 : 0;
    RPCA_LAUNCH(c, prof, RPCA_PHASE_VPASS,
                h ? launch_vpass_h(q, mode, Ucons, c->U[c->cur ^ 1], c->V[c->vcur], fin, x3, st)
                  : launch_vpass(q, mode, Ucons, 0, c->U[c->cur ^ 1], c->V[c->vcur], fin, st),
                "V-pass launch");
    RPCA_LAUNCH(c, prof, RPCA_PHASE_VFINAL, launch_vfinal(q, c->Ginv, 0, fin ? 1 : 0, st),
                "V finish launch");
    if (p.u_mode == RPCA_U_CLOSED)
      RPCA_LAUNCH(c, prof, RPCA_PHASE_CLIENT_FACTOR, launch_client_factor(q, st), "client factor launch");
    RPCA_LAUNCH(c, prof, RPCA_PHASE_SPASS,
                h ? launch_spass_h(q, Ucons, x3, st) : launch_spass(q, Ucons, 0, nullptr, 0, 0, 0, p.E, st),
                "S-pass launch");
    RPCA_LAUNCH(c, prof, RPCA_PHASE_UUPDATE, launch_uupdate(q, c->U[c->cur ^ 1], 0, Ucons, 1, st),
                "U update launch");
    c->fin_pending = true;
    c->vcur = vn;
    c->cur ^= 1;
    c->rounds += 1;
    c->p.lam_rec = c->p.lam;
    c->sparse_valid = q.Smask != nullptr;
    return RPCA_OK;
  }
  for (int k = 0; k < p.K; ++k) {
    const float* Uin = k == 0 ? Ucons : c->Uc[(k - 1) & 1];
    const int64_t us = k == 0 ? 0 : ustride;
    const double* Gin = k == 0 ? c->Ginv : c->Ginv + gstride;
    const int64_t gs = k == 0 ? 0 : gstride;
    for (int qi = 0; qi < c->inner; ++qi) {
      const int vn = c->vcur ^ 1;
      const DevParams q = with_v(c, vn);
      RPCA_HIP(c, unfold_finalize(c, prof), "finalize launch");
      double* fin = c->fin_pending ? c->Ginv : nullptr;
      c->fin_pending = false;
      RPCA_LAUNCH(c, prof, RPCA_PHASE_VPASS,
                  launch_vpass(q, kSStored, Uin, us, nullptr, nullptr, fin, st), "V-pass launch");
      RPCA_LAUNCH(c, prof, RPCA_PHASE_VFINAL, launch_vfinal(q, Gin, gs, fin ? 1 : 0, st),
                  "V finish launch");
      c->vcur = vn;
      if (p.u_mode == RPCA_U_CLOSED && qi == c->inner - 1)
        RPCA_LAUNCH(c, prof, RPCA_PHASE_CLIENT_FACTOR, launch_client_factor(q, st), "client factor launch");
      RPCA_LAUNCH(c, prof, RPCA_PHASE_SPASS, launch_spass(q, Uin, us, p.S, p.lds, 0, 0, p.E, st), "S-pass launch");
    }
    if (k == p.K - 1) {
      RPCA_LAUNCH(c, prof, RPCA_PHASE_UUPDATE, launch_uupdate(p, c->U[c->cur ^ 1], 0, Ucons, 1, st),
                  "U update launch");
      c->fin_pending = true;
    } else {
      RPCA_LAUNCH(c, prof, RPCA_PHASE_UUPDATE, launch_uupdate(p, c->Uc[k & 1], ustride, nullptr, 0, st),
                  "U update launch");
      RPCA_LAUNCH(c, prof, RPCA_PHASE_FINALIZE, launch_finalize(p, c->Ginv + gstride, gstride, 1, 0, st),
                  "finalize launch");
    }
  }
  c->cur ^= 1;
  c->rounds += 1;
  c->p.lam_rec = c->p.lam;
  return RPCA_OK;
}

}  // namespace

namespace {

rpca_status guard(rpca_ctx* c) {
  if (!c) return RPCA_EINVAL;
  if (c->poisoned) return RPCA_ESTATE;
  return RPCA_OK;
}

// Run a deferred finalize now (before reading statistics or the Gram inverse).
rpca_status flush_finalize(rpca_ctx* c) {
  if (c->fin_pending) {
    RPCA_HIP(c, launch_finalize(c->p, c->Ginv, 0, 0, 1, c->stream), "finalize launch");
    c->fin_pending = false;
  }
  return RPCA_OK;
}

// ||U V^T - X2 Y2^T||_F^2 and ||X2 Y2^T||_F^2 into c->dout (device).
rpca_status enqueue_distance(rpca_ctx* c, const float* X2, const float* Y2, int rp2) {
  RPCA_HIP(c,
           launch_factor_distance(c->p, c->U[c->cur], v_fb(c->V[c->vcur], c->p.NVP, c->p.RP), c->p.RP, X2, Y2, rp2, c->dpart,
                                  c->dpart2, c->dout, c->stream),
           "factor distance launch");
  return RPCA_OK;
}

}  // namespace

extern "C" {

const char* rpca_params_error(const rpca_params* p) { return check_params(p); }

rpca_status rpca_workspace_bytes(const rpca_params* p, size_t* bytes) {
  if (check_params(p) || !bytes) return RPCA_EINVAL;
  *bytes = make_layout(p).total;
  return RPCA_OK;
}

rpca_status rpca_init(rpca_ctx** out, const rpca_params* prm, const float* const* M_blocks,
                      const int64_t* ldm, const float* U0, int64_t ldu, void* workspace,
                      size_t ws_bytes, void* stream) {
  g_init_err.clear();
  if (!out) return init_fail(RPCA_EINVAL, "out is NULL");
  *out = nullptr;
  if (const char* msg = check_params(prm)) return init_fail(RPCA_EINVAL, msg);
  if (!M_blocks || !ldm) return init_fail(RPCA_EINVAL, "M_blocks or ldm is NULL");
  if (U0 && ldu < prm->m) return init_fail(RPCA_EINVAL, "ldu < m");
  for (int i = 0; i < prm->E; ++i) {
    // Kernels address 16 columns of a block with 32-bit byte offsets.
    if (!M_blocks[i] || ldm[i] < prm->m || ldm[i] % 4 != 0 || ldm[i] >= ((int64_t)1 << 26) ||
        reinterpret_cast<uintptr_t>(M_blocks[i]) % 16 != 0)
      return init_fail(RPCA_EINVAL, "M block " + std::to_string(i) +
                                        ": NULL, not 16-byte aligned, or ldm not a multiple of 4 "
                                        "in [m, 2^26)");
  }
  const Layout L = make_layout(prm);
  if (!workspace) return init_fail(RPCA_EWORKSPACE, "workspace is NULL");
  if (ws_bytes < L.total)
    return init_fail(RPCA_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) +
                                          " bytes; these parameters need " +
                                          std::to_string(L.total));
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return init_fail(RPCA_EWORKSPACE, "workspace is not 256-byte aligned");

  if ((prm->flags & RPCA_FLAG_GRAPH) && !stream)
    return init_fail(RPCA_EINVAL, "RPCA_FLAG_GRAPH needs a stream other than the null stream");
  if (prm->flags & RPCA_FLAG_BF16X3)
    for (int i = 0; i < prm->E; ++i)
      if (ldm[i] >= ((int64_t)1 << 24))
        return init_fail(RPCA_EINVAL, "RPCA_FLAG_BF16X3 needs every ldm < 2^24");
  rpca_ctx* c = new rpca_ctx();
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->inner = prm->inner;
  char* ws = static_cast<char*>(workspace);
  c->ws = ws;
  c->ws_bytes = L.total;
  c->own_ranges = {{L.clients, (size_t)prm->E * sizeof(ClientDev)},
                   {L.clients_lpt, (size_t)prm->E * sizeof(ClientDev)},
                   {L.vg64, (size_t)L.ng64 * sizeof(VTile)},
                   {L.Mbv, L.Mbs - L.Mbv},
                   {L.Mbs, L.Wpart - L.Mbs}};
  std::sort(c->own_ranges.begin(), c->own_ranges.end());
  c->widths.assign(prm->n_cols, prm->n_cols + prm->E);
  DevParams& p = c->p;
  p.m = (int32_t)prm->m;
  p.MP = L.MP;
  p.r = prm->r;
  p.RP = L.RP;
  p.NS = L.NS;
  p.E = prm->E;
  p.K = prm->K;
  p.NVP = L.NVP;
  p.n = L.n;
  p.lds = L.lds;
  p.nrb = L.nrb;
  p.nub = L.nub;
  p.ngroups = L.ngroups;
  p.ng64 = L.ng64;
  p.vsplit = L.vsplit;
  p.vsplit_rows = L.vsplit_rows;
  // Shared-operand V-pass waves pay off once a chunk's U operands cost more
  // loads than its M (the rebuild's NS packed rank steps); the autotuner
  // revisits this.
  // (Ranks above 64 take one group per wave.)
  p.vcols = L.NS > 5 && L.RP <= kFoldMaxRP ? 4 : 1;
  // S-pass work-groups of 8 waves, two per 32-row strip taking alternate
  // column chunks; the autotuner also tries one wave per strip. (Ranks above
  // 64 take one wave per strip.)
  p.sphases = L.RP <= kFoldMaxRP ? 2 : 1;
  c->vsplit_max = L.vsplit_max;
  p.u_mode = prm->u_mode;
  p.eta_sched = prm->eta_sched;
  p.lam = (float)prm->lambda;
  p.lam_rec = p.lam;
  p.lam_target = p.lam;
  p.huber = 0;
  p.omega = 1.0;
  p.rho = prm->rho;
  p.eta0 = prm->eta0;
  p.bf16 = L.bf16 ? 1 : 0;
  p.RK = L.RK;
  p.NK = L.RK / 32;
  p.Mbv = L.mcopy ? reinterpret_cast<uint16_t*>(ws + L.Mbv) : nullptr;
  p.Mbs = L.mcopy ? reinterpret_cast<uint16_t*>(ws + L.Mbs) : nullptr;
  c->prec = L.mcopy ? RPCA_PREC_BF16 : L.bf16 ? RPCA_PREC_BF16X3 : RPCA_PREC_FP32;
  for (int i = 0; i < prm->E; ++i) c->max_ldm = std::max(c->max_ldm, ldm[i]);
  p.clients = reinterpret_cast<const ClientDev*>(ws + L.clients);
  p.clients_lpt = reinterpret_cast<const ClientDev*>(ws + L.clients_lpt);
  p.vgroups = reinterpret_cast<const VGroup*>(ws + L.vgroups);
  p.vg64 = reinterpret_cast<const VTile*>(ws + L.vg64);
  p.S = L.recompute ? nullptr : reinterpret_cast<float*>(ws + L.S);
  const bool sparse = (prm->flags & RPCA_FLAG_SPARSE_S) != 0;
  p.Smask = sparse ? reinterpret_cast<uint64_t*>(ws + L.Smask) : nullptr;
  p.Sval = sparse ? reinterpret_cast<float*>(ws + L.Sval) : nullptr;
  c->recompute = L.recompute;
  c->use_graph = L.recompute && (prm->flags & RPCA_FLAG_GRAPH);
  c->V[0] = reinterpret_cast<float*>(ws + L.V0);
  c->V[1] = reinterpret_cast<float*>(ws + L.V1);
  p.V = c->V[0];
  p.ublock = fb_floats(L.MP, L.RP, L.NS);
  p.Wpart = reinterpret_cast<float*>(ws + L.Wpart);
  p.P = reinterpret_cast<float*>(ws + L.P);
  p.gv_part = reinterpret_cast<double*>(ws + L.gv);
  p.gv_tr = reinterpret_cast<double*>(ws + L.gvtr);
  p.Afac = reinterpret_cast<double*>(ws + L.Af);
  p.gram_part = reinterpret_cast<double*>(ws + L.gram);
  p.spart = reinterpret_cast<double*>(ws + L.spart);
  p.upart = reinterpret_cast<double*>(ws + L.upart);
  p.ucl_sq = reinterpret_cast<double*>(ws + L.ucl);
  p.dstate = reinterpret_cast<DevState*>(ws + L.dstate);
  p.hist = reinterpret_cast<StatsRec*>(ws + L.hist);
  p.stat_part = reinterpret_cast<double*>(ws + L.stat_part);
  p.queue = reinterpret_cast<uint32_t*>(ws + L.queue);
  p.vqueue = 0;
  p.squeue = 0;
  c->use_sparse = p.Smask ? 1 : 0;
  c->U[0] = reinterpret_cast<float*>(ws + L.U0);
  c->U[1] = reinterpret_cast<float*>(ws + L.U1);
  c->Uc[0] = reinterpret_cast<float*>(ws + L.Uc0);
  c->Uc[1] = reinterpret_cast<float*>(ws + L.Uc1);
  c->Ginv = reinterpret_cast<double*>(ws + L.Ginv);
  c->Uprev = reinterpret_cast<float*>(ws + L.Uprev);
  c->Vprev = reinterpret_cast<float*>(ws + L.Vprev);
  c->Ut = reinterpret_cast<float*>(ws + L.Ut);
  c->Vt = reinterpret_cast<float*>(ws + L.Vt);
  c->dpart = reinterpret_cast<double*>(ws + L.dpart);
  c->dpart2 = reinterpret_cast<double*>(ws + L.dpart2);
  c->dout = reinterpret_cast<double*>(ws + L.dout);

  // Client table (Section 2.1: client i holds columns [col_off[i], col_off[i+1])).
  c->clients.resize(prm->E);
  c->col_off.resize(prm->E + 1);
  int64_t col = 0, vrow = 0;
  int32_t g = 0;
  for (int i = 0; i < prm->E; ++i) {
    ClientDev& cd = c->clients[i];
    const int32_t ni = (int32_t)prm->n_cols[i];
    cd.M = M_blocks[i];
    cd.ldm = ldm[i];
    cd.s_off = L.lds * col;
    cd.col0 = col;
    cd.n = ni;
    cd.vrow0 = (int32_t)vrow;
    cd.g0 = g;
    for (int32_t j0 = 0; j0 < ni; j0 += kVCols) {
      c->vgroups.push_back(VGroup{i, j0, ni - j0 < kVCols ? ni - j0 : kVCols, (int32_t)vrow + j0});
      ++g;
    }
    cd.g1 = g;
    cd.c = prm->rho * (double)ni / (double)L.n;
    cd.idx = i;
    cd.pad = 0;
    for (int32_t j0 = 0; j0 < ni; j0 += kVStreamCols)
      c->vg64.push_back(VTile{cd, i, j0, ni - j0 < kVStreamCols ? ni - j0 : kVStreamCols, 0});
    c->col_off[i] = col;
    col += ni;
    vrow += round_up(ni, kVPad);
  }
  c->col_off[prm->E] = col;
  c->clients_lpt = c->clients;
  std::stable_sort(c->clients_lpt.begin(), c->clients_lpt.end(),
                   [](const ClientDev& x, const ClientDev& y) { return x.n > y.n; });

  hipStream_t st = c->stream;
  hipError_t e = hipMemsetAsync(workspace, 0, L.total, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.clients, c->clients.data(), c->clients.size() * sizeof(ClientDev),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.clients_lpt, c->clients_lpt.data(),
                       c->clients_lpt.size() * sizeof(ClientDev), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.vgroups, c->vgroups.data(), c->vgroups.size() * sizeof(VGroup),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.vg64, c->vg64.data(), c->vg64.size() * sizeof(VTile),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = U0 ? launch_copy_in_U(p, U0, ldu, c->U[0], st) : launch_init_U_gauss(p, prm->seed, c->U[0], st);
  if (e == hipSuccess && L.mcopy) e = launch_m_to_bf16(p, st);
  if (e == hipSuccess) e = launch_gram_init(p, c->U[0], st);
  if (e == hipSuccess) e = launch_finalize(p, c->Ginv, 0, 0, 0, st);
  // The host tables must outlive the asynchronous copies above.
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete c;
    return init_fail(RPCA_EDEVICE, std::string("initialisation: ") + hipGetErrorString(e));
  }
  *out = c;
  const double mn = (double)prm->m * (double)L.n;
  if (prm->rho * prm->rho > prm->lambda * prm->lambda * mn) {
    c->err = "rho^2 > lambda^2 m n: only U = 0 is stationary (Theorem 2)";
    return RPCA_WARN_THM2;
  }
  return RPCA_OK;
}

}  // extern "C"

// The static workspace of rpca_init_static: one array per GPU (each device's
// code object holds its own copy), at most one live context per GPU. Host code
// never passes the array's name to a kernel or a HIP call: the name is a
// host-side stand-in, and the device address comes from hipGetSymbolAddress,
// taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[RPCA_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
rpca_ctx* g_static_owner[kMaxDevices] = {};
}  // namespace

extern "C" {

rpca_status rpca_init_static(rpca_ctx** out, const rpca_params* prm, const float* const* M_blocks,
                             const int64_t* ldm, const float* U0, int64_t ldu, void* stream) {
  g_init_err.clear();
  if (!out) return init_fail(RPCA_EINVAL, "out is NULL");
  *out = nullptr;
  if (const char* msg = check_params(prm)) return init_fail(RPCA_EINVAL, msg);
  const size_t need = make_layout(prm).total;
  if (need > RPCA_STATIC_WORKSPACE_BYTES)
    return init_fail(RPCA_EWORKSPACE, "these parameters need " + std::to_string(need) +
                                          " bytes of workspace; the static workspace holds " +
                                          std::to_string(RPCA_STATIC_WORKSPACE_BYTES));
  int dev = -1;
  const hipError_t ed = hipGetDevice(&dev);
  if (ed != hipSuccess) return init_fail(RPCA_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(ed));
  if (dev < 0 || dev >= kMaxDevices)
    return init_fail(RPCA_EINVAL, "device index beyond the library's table of " +
                                      std::to_string(kMaxDevices));
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (g_static_owner[dev])
    return init_fail(RPCA_ESTATE, "another context uses this GPU's static workspace; destroy it first");
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return init_fail(RPCA_EDEVICE, std::string("hipGetSymbolAddress of the static workspace: ") +
                                         hipGetErrorString(e));
    g_static_ptr[dev] = ptr;
  }
  const rpca_status st = rpca_init(out, prm, M_blocks, ldm, U0, ldu, g_static_ptr[dev],
                                   RPCA_STATIC_WORKSPACE_BYTES, stream);
  if (st >= 0 && *out) {
    (*out)->static_dev = dev;
    g_static_owner[dev] = *out;
  }
  return st;
}

// Two rounds from a steady state (rebuilt S, finalize deferred) as one graph
// launch; the graph for this buffer parity is captured on first use. The host
// state after two rounds equals the state before them except for the count.
rpca_status enqueue_round_pair_graph(rpca_ctx* c) {
  const int key = c->cur;
  if (!c->gexec[key]) {
    const int cur = c->cur, vcur = c->vcur;
    const int64_t rounds = c->rounds;
    const bool fin = c->fin_pending;
    RPCA_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    rpca_status s1 = enqueue_round(c);
    rpca_status s2 = s1 == RPCA_OK ? enqueue_round(c) : s1;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->cur = cur;
    c->vcur = vcur;
    c->rounds = rounds;
    c->fin_pending = fin;
    if (s2 != RPCA_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s2;
    }
    RPCA_HIP(c, e, "end capture");
    const hipError_t ei = hipGraphInstantiate(&c->gexec[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    RPCA_HIP(c, ei, "graph instantiate");
  }
  RPCA_HIP(c, hipGraphLaunch(c->gexec[key], c->stream), "graph launch");
  c->rounds += 2;
  return RPCA_OK;
}

rpca_status rpca_step(rpca_ctx* c, int32_t rounds) {
  if (rpca_status s = guard(c)) return s;
  if (rounds < 0) return fail(c, RPCA_EINVAL, "rounds must be >= 0");
  int32_t t = 0;
  while (t < rounds) {
    // A graph bakes its launches' parameters, including the lambda the first
    // round's deferred record uses: capture only in a steady state, where
    // that is the lambda of every round.
    // With sparse S the graph's first round reads the sparse S, which must
    // then be there.
    const bool sparse_ok =
        !c->p.Smask || !c->use_sparse || c->prec != RPCA_PREC_FP32 || c->sparse_valid;
    if (c->use_graph && rounds - t >= 2 && c->rounds >= 1 && c->fin_pending &&
        c->p.lam_rec == c->p.lam && sparse_ok) {
      if (rpca_status s = enqueue_round_pair_graph(c)) return s;
      t += 2;
    } else {
      if (rpca_status s = enqueue_round(c)) return s;
      t += 1;
    }
  }
  return RPCA_OK;
}

// Graphs captured before bake the old launch shapes and kernels.
static void drop_graphs(rpca_ctx* c) {
  for (hipGraphExec_t& g : c->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Row splits for a given count: rows per split a multiple of 16 (32 when BF16
// rounds, which walk 32-row chunks, may run).
static void set_vsplit(rpca_ctx* c, int64_t vs) {
  const int64_t m = c->p.m;
  const int64_t rows = round_up((m + vs - 1) / vs, c->p.bf16 ? 32 : 16);
  c->p.vsplit_rows = (int32_t)rows;
  c->p.vsplit = (int32_t)((m + rows - 1) / rows);
}

static rpca_launch_shape shape_of(const rpca_ctx* c) {
  return rpca_launch_shape{c->p.vsplit, c->p.vcols, c->p.sphases, c->p.vqueue, c->p.squeue,
                           c->use_sparse};
}

static void apply_shape(rpca_ctx* c, const rpca_launch_shape& k) {
  set_vsplit(c, k.vsplit);
  c->p.vcols = k.vcols;
  c->p.sphases = k.sphases;
  c->p.vqueue = k.vqueue;
  c->p.squeue = k.squeue;
  c->use_sparse = c->p.Smask ? k.sparse : 0;
}

static bool same_shape(const rpca_launch_shape& a, const rpca_launch_shape& b) {
  return a.vsplit == b.vsplit && a.vcols == b.vcols && a.sphases == b.sphases &&
         a.vqueue == b.vqueue && a.squeue == b.squeue && a.sparse == b.sparse;
}

rpca_status rpca_autotune(rpca_ctx* c, int32_t rounds, rpca_launch_shape* out) {
  if (rpca_status s = guard(c)) return s;
  if (rounds < 1) return fail(c, RPCA_EINVAL, "rounds must be >= 1");
  const rpca_launch_shape start = shape_of(c);
  hipEvent_t a = nullptr, b = nullptr;
  RPCA_HIP(c, hipEventCreate(&a), "event");
  const hipError_t eb = hipEventCreate(&b);
  if (eb != hipSuccess) {
    (void)hipEventDestroy(a);
    return dev_fail(c, eb, "event");
  }
  rpca_status result = RPCA_OK;
  // Milliseconds of `rounds` rounds at shape k, after one untimed round; < 0
  // on failure (result set).
  auto time_shape = [&](const rpca_launch_shape& k) -> float {
    apply_shape(c, k);
    if ((result = enqueue_round(c)) != RPCA_OK) return -1.f;
    hipError_t e = hipEventRecord(a, c->stream);
    for (int32_t t = 0; t < rounds && e == hipSuccess && result == RPCA_OK; ++t)
      result = enqueue_round(c);
    if (result != RPCA_OK) return -1.f;
    if (e == hipSuccess) e = hipEventRecord(b, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) {
      result = dev_fail(c, e, "autotune timing");
      return -1.f;
    }
    return ms;
  };
  // Stage 1, the V-pass: (row splits, column groups per wave) at the current
  // S-pass shape.
  std::vector<rpca_launch_shape> cand;
  const int64_t v0 = start.vsplit;
  for (int64_t v : {(v0 + 1) / 2, v0, 2 * v0, 3 * v0, 4 * v0, (int64_t)c->vsplit_max}) {
    if (v < 1 || v > c->vsplit_max) continue;
    set_vsplit(c, v);
    for (int32_t g : {1, 4}) {
      if (g == 4 && c->p.RP > kFoldMaxRP) continue;
      const rpca_launch_shape k{c->p.vsplit, g, start.sphases, start.vqueue, start.squeue,
                                start.sparse};
      if (std::none_of(cand.begin(), cand.end(), [&](const rpca_launch_shape& x) { return same_shape(x, k); }))
        cand.push_back(k);
    }
  }
  // Two passes over the candidates, times summed: the candidates differ by a
  // few percent of a round, about the drift of one timing.
  rpca_launch_shape best = start;
  std::vector<float> tot(cand.size(), 0.f);
  for (int rep = 0; rep < 2 && result == RPCA_OK; ++rep)
    for (size_t q = 0; q < cand.size() && result == RPCA_OK; ++q) {
      const float ms = time_shape(cand[q]);
      if (ms >= 0.f) tot[q] += ms;
    }
  if (result == RPCA_OK && !cand.empty())
    best = cand[std::min_element(tot.begin(), tot.end()) - tot.begin()];
  // Stage 2, the S-pass at the chosen V-pass shape: in FP32 rounds two
  // column phases and one; in BF16 rounds the register form (two phases)
  // and the LDS-staged form (one). Timed in turn twice each (the gap is a
  // few percent of a round; three-product rounds have one form).
  if (result == RPCA_OK && (c->prec == RPCA_PREC_FP32 || c->prec == RPCA_PREC_BF16) &&
      c->p.RP <= kFoldMaxRP) {
    const std::vector<rpca_launch_shape> ks = {
        {best.vsplit, best.vcols, 2, best.vqueue, best.squeue, best.sparse},
        {best.vsplit, best.vcols, 1, best.vqueue, best.squeue, best.sparse}};
    std::vector<float> ts(ks.size(), 0.f);
    for (int rep = 0; rep < 2 && result == RPCA_OK; ++rep)
      for (size_t q = 0; q < ks.size() && result == RPCA_OK; ++q) {
        const float ms = time_shape(ks[q]);
        if (ms >= 0.f) ts[q] += ms;
      }
    if (result == RPCA_OK)
      best = ks[std::min_element(ts.begin(), ts.end()) - ts.begin()];
  }
  // Stage 3, the launch form of both passes at the chosen shapes: one
  // work-group per tile, or a persistent launch over a tile queue, for each.
  if (result == RPCA_OK) {
    std::vector<rpca_launch_shape> ks;
    for (int32_t vq : {0, 1})
      for (int32_t sq : {0, 1})
        ks.push_back({best.vsplit, best.vcols, best.sphases, vq, sq, best.sparse});
    std::vector<float> ts(ks.size(), 0.f);
    for (int rep = 0; rep < 2 && result == RPCA_OK; ++rep)
      for (size_t q = 0; q < ks.size() && result == RPCA_OK; ++q) {
        const float ms = time_shape(ks[q]);
        if (ms >= 0.f) ts[q] += ms;
      }
    if (result == RPCA_OK)
      best = ks[std::min_element(ts.begin(), ts.end()) - ts.begin()];
  }
  // Stage 4, with RPCA_FLAG_SPARSE_S and FP32 rounds: S handed over in sparse
  // form or rebuilt, each tuned anew for the V-pass form (which of the two
  // pays depends on r and on how dense S is). Every timing starts with an
  // untimed round, which also refills the sparse S after a rebuilt round.
  if (result == RPCA_OK && c->p.Smask && c->prec == RPCA_PREC_FP32) {
    std::vector<rpca_launch_shape> ks;
    for (int32_t sp : {0, 1})
      for (int32_t vq : {0, 1})
        ks.push_back({best.vsplit, best.vcols, best.sphases, vq, best.squeue, sp});
    std::vector<float> ts(ks.size(), 0.f);
    for (int rep = 0; rep < 2 && result == RPCA_OK; ++rep)
      for (size_t q = 0; q < ks.size() && result == RPCA_OK; ++q) {
        const float ms = time_shape(ks[q]);
        if (ms >= 0.f) ts[q] += ms;
      }
    if (result == RPCA_OK)
      best = ks[std::min_element(ts.begin(), ts.end()) - ts.begin()];
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (result != RPCA_OK) best = start;
  apply_shape(c, best);
  drop_graphs(c);
  if (out) *out = shape_of(c);
  return result;
}

rpca_status rpca_get_launch_shape(rpca_ctx* c, rpca_launch_shape* out) {
  if (rpca_status s = guard(c)) return s;
  if (!out) return fail(c, RPCA_EINVAL, "out is NULL");
  *out = shape_of(c);
  return RPCA_OK;
}

rpca_status rpca_set_launch_shape(rpca_ctx* c, const rpca_launch_shape* k) {
  if (rpca_status s = guard(c)) return s;
  if (!k) return fail(c, RPCA_EINVAL, "shape is NULL");
  if (k->vsplit < 1 || k->vsplit > c->vsplit_max)
    return fail(c, RPCA_EINVAL, "row splits must lie in [1, " + std::to_string(c->vsplit_max) + "]");
  if (k->vcols != 1 && k->vcols != 4)
    return fail(c, RPCA_EINVAL, "column groups per V-pass wave must be 1 or 4");
  if (k->sphases != 1 && k->sphases != 2)
    return fail(c, RPCA_EINVAL, "S-pass column phases must be 1 or 2");
  if ((k->vqueue != 0 && k->vqueue != 1) || (k->squeue != 0 && k->squeue != 1))
    return fail(c, RPCA_EINVAL, "launch forms must be 0 (one work-group per tile) or 1 (tile queue)");
  if (k->sparse != 0 && k->sparse != 1)
    return fail(c, RPCA_EINVAL, "sparse must be 0 (rebuild S) or 1 (sparse S)");
  if (k->sparse && !c->p.Smask)
    return fail(c, RPCA_EINVAL, "sparse S needs a context created with RPCA_FLAG_SPARSE_S");
  if (c->p.RP > kFoldMaxRP && (k->vcols != 1 || k->sphases != 1))
    return fail(c, RPCA_EINVAL,
                "ranks above 64 take 1 column group per V-pass wave and 1 S-pass column phase");
  apply_shape(c, *k);
  drop_graphs(c);
  return RPCA_OK;
}

rpca_status rpca_copy_state(rpca_ctx* dst, rpca_ctx* src) {
  if (rpca_status s = guard(dst)) return s;
  if (rpca_status s = guard(src)) return s;
  if (dst == src) return RPCA_OK;
  const DevParams &a = dst->p, &b = src->p;
  if (dst->ws_bytes != src->ws_bytes || dst->widths != src->widths || a.m != b.m || a.r != b.r ||
      a.K != b.K || a.u_mode != b.u_mode || a.bf16 != b.bf16 || a.eta_sched != b.eta_sched ||
      a.rho != b.rho || a.eta0 != b.eta0 || dst->inner != src->inner ||
      dst->recompute != src->recompute || (a.Smask == nullptr) != (b.Smask == nullptr))
    return fail(dst, RPCA_EINVAL, "rpca_copy_state needs contexts created with the same parameters");
  RPCA_HIP(src, hipStreamSynchronize(src->stream), "synchronize");
  size_t at = 0;
  for (const auto& rg : dst->own_ranges) {
    if (rg.first > at)
      RPCA_HIP(dst, hipMemcpyAsync(dst->ws + at, src->ws + at, rg.first - at, hipMemcpyDeviceToDevice,
                                   dst->stream), "copy state");
    at = std::max(at, rg.first + rg.second);
  }
  if (dst->ws_bytes > at)
    RPCA_HIP(dst, hipMemcpyAsync(dst->ws + at, src->ws + at, dst->ws_bytes - at,
                                 hipMemcpyDeviceToDevice, dst->stream), "copy state");
  dst->rounds = src->rounds;
  dst->cur = src->cur;
  dst->vcur = src->vcur;
  dst->fin_pending = src->fin_pending;
  dst->have_prev = src->have_prev;
  dst->sparse_valid = src->sparse_valid;
  dst->have_target = src->have_target;
  dst->RPT = src->RPT;
  dst->prec = src->prec;
  dst->p.lam = src->p.lam;
  dst->p.lam_rec = src->p.lam_rec;
  dst->p.omega = src->p.omega;
  dst->p.vsplit = src->p.vsplit;
  dst->p.vsplit_rows = src->p.vsplit_rows;
  dst->p.vcols = src->p.vcols;
  dst->p.sphases = src->p.sphases;
  dst->p.vqueue = src->p.vqueue;
  dst->p.squeue = src->p.squeue;
  drop_graphs(dst);
  return RPCA_OK;
}

rpca_status rpca_set_lambda(rpca_ctx* c, double lambda) {
  if (rpca_status s = guard(c)) return s;
  if (!(lambda >= 0.0) || !std::isfinite(lambda))
    return fail(c, RPCA_EINVAL, "lambda must be finite and >= 0");
  if (!c->recompute)
    return fail(c, RPCA_EINVAL, "rpca_set_lambda needs K = 1, inner = 1 and no RPCA_FLAG_STORE_S");
  if ((float)lambda != c->p.lam) drop_graphs(c);
  c->p.lam = (float)lambda;
  return RPCA_OK;
}

rpca_status rpca_set_step(rpca_ctx* c, double omega) {
  if (rpca_status s = guard(c)) return s;
  if (!(omega > 0.0) || !(omega <= 4.0))
    return fail(c, RPCA_EINVAL, "the step multiplier must lie in (0, 4]");
  if (omega != c->p.omega) drop_graphs(c);
  c->p.omega = omega;
  return RPCA_OK;
}

rpca_status rpca_set_precision(rpca_ctx* c, int32_t precision) {
  if (rpca_status s = guard(c)) return s;
  if (precision != RPCA_PREC_FP32 && precision != RPCA_PREC_BF16 && precision != RPCA_PREC_BF16X3)
    return fail(c, RPCA_EINVAL, "unknown precision");
  if (precision == RPCA_PREC_BF16 && !c->p.Mbv)
    return fail(c, RPCA_EINVAL, "BF16 rounds need a context created with RPCA_FLAG_BF16");
  if (precision == RPCA_PREC_BF16X3 && !c->p.bf16)
    return fail(c, RPCA_EINVAL,
                "three-product BF16 rounds need RPCA_FLAG_BF16X3 or RPCA_FLAG_BF16");
  if (precision == RPCA_PREC_BF16X3 && c->max_ldm >= ((int64_t)1 << 24))
    return fail(c, RPCA_EINVAL, "three-product BF16 rounds need every ldm < 2^24");
  if (precision != c->prec) drop_graphs(c);
  c->prec = precision;
  return RPCA_OK;
}

rpca_status rpca_set_target(rpca_ctx* c, const float* Ustar, int64_t ldus, const float* Vstar,
                            int64_t ldvs, int32_t rstar) {
  if (rpca_status s = guard(c)) return s;
  if (!Ustar || !Vstar || rstar < 1 || rstar > kMaxRank || ldus < c->p.m || ldvs < c->p.n)
    return fail(c, RPCA_EINVAL, "invalid target factors");
  c->RPT = (int)round_up(rstar, 16);
  RPCA_HIP(c,
           launch_pack_target(c->p, c->clients.data(), c->col_off.data(), Ustar, ldus, Vstar,
                              ldvs, rstar, c->Ut, c->Vt, c->RPT, c->stream),
           "target pack launch");
  c->have_target = true;
  return RPCA_OK;
}

rpca_status rpca_target_error(rpca_ctx* c, double* relerr) {
  if (rpca_status s = guard(c)) return s;
  if (!relerr) return fail(c, RPCA_EINVAL, "relerr is NULL");
  if (!c->have_target) {
    *relerr = NAN;
    return RPCA_OK;
  }
  if (rpca_status s = enqueue_distance(c, c->Ut, c->Vt, c->RPT)) return s;
  double h[2];
  RPCA_HIP(c, hipMemcpyAsync(h, c->dout, sizeof(h), hipMemcpyDeviceToHost, c->stream), "copy");
  RPCA_HIP(c, hipStreamSynchronize(c->stream), "synchronize");
  *relerr = std::sqrt(std::fmax(h[0], 0.0) / h[1]);
  return RPCA_OK;
}

rpca_status rpca_solve(rpca_ctx* c, int32_t max_rounds, double tol, int32_t check_every,
                       int32_t* rounds_done, double* metric) {
  if (rpca_status s = guard(c)) return s;
  if (max_rounds < 0 || check_every < 1) return fail(c, RPCA_EINVAL, "bad solve arguments");
  int32_t done = 0;
  double last = INFINITY;
  const size_t ubytes = (size_t)c->p.RP * c->p.MP * sizeof(float);
  const size_t vbytes = (size_t)c->p.RP * c->p.NVP * sizeof(float);
  rpca_status result = RPCA_OK;
  while (done < max_rounds) {
    const int32_t nr = max_rounds - done < check_every ? max_rounds - done : check_every;
    if (rpca_status s = rpca_step(c, nr)) return s;
    done += nr;
    bool have_metric = false;
    if (c->have_target) {
      if (rpca_status s = enqueue_distance(c, c->Ut, c->Vt, c->RPT)) return s;
      have_metric = true;
    } else if (c->have_prev) {
      if (rpca_status s = enqueue_distance(c, c->Uprev, c->Vprev, c->p.RP)) return s;
      have_metric = true;
    }
    if (!c->have_target) {
      RPCA_HIP(c, hipMemcpyAsync(c->Uprev, c->U[c->cur], ubytes, hipMemcpyDeviceToDevice, c->stream),
               "copy U");
      RPCA_HIP(c, hipMemcpyAsync(c->Vprev, v_fb(c->V[c->vcur], c->p.NVP, c->p.RP), vbytes, hipMemcpyDeviceToDevice, c->stream),
               "copy V");
      c->have_prev = true;
    }
    if (rpca_status s = flush_finalize(c)) return s;
    double h[2] = {0.0, 1.0};
    StatsRec rec;
    if (have_metric)
      RPCA_HIP(c, hipMemcpyAsync(h, c->dout, sizeof(h), hipMemcpyDeviceToHost, c->stream), "copy");
    RPCA_HIP(c,
             hipMemcpyAsync(&rec, c->p.hist + (c->rounds - 1) % kHist, sizeof(rec),
                            hipMemcpyDeviceToHost, c->stream),
             "copy stats");
    RPCA_HIP(c, hipStreamSynchronize(c->stream), "synchronize");
    if (!std::isfinite(rec.objective)) {
      result = fail(c, RPCA_ENONFINITE, "non-finite objective");
      break;
    }
    if (have_metric) {
      last = h[1] > 0.0 ? std::sqrt(std::fmax(h[0], 0.0) / h[1]) : INFINITY;
      if (last <= tol) break;
    }
  }
  if (rounds_done) *rounds_done = done;
  if (metric) *metric = last;
  return result;
}

rpca_status rpca_get_LS(rpca_ctx* c, int32_t client, float* L, int64_t ldl, float* S,
                        int64_t lds) {
  if (rpca_status s = guard(c)) return s;
  if (client < -1 || client >= c->p.E) return fail(c, RPCA_EINVAL, "client out of range");
  if ((L && ldl < c->p.m) || (S && lds < c->p.m)) return fail(c, RPCA_EINVAL, "leading dimension < m");
  const int b = client < 0 ? 0 : client, e = client < 0 ? c->p.E : client + 1;
  const DevParams q = with_v(c, c->vcur);
  const bool emit_s = S && c->recompute;
  if (L || (S && !c->recompute))
    RPCA_HIP(c,
             launch_materialize(q, c->clients.data(), c->col_off.data(), c->U[c->cur], b, e, L,
                                ldl, c->recompute ? nullptr : S, lds, c->stream),
             "materialize launch");
  if (emit_s) {
    if (c->rounds == 0) {
      // No round has run: S^(0) = 0.
      for (int i = b; i < e; ++i)
        RPCA_HIP(c,
                 hipMemset2DAsync(S + (c->col_off[i] - c->col_off[b]) * lds, lds * sizeof(float), 0,
                                  c->p.m * sizeof(float), c->clients[i].n, c->stream),
                 "zero S");
    } else {
      // S of the last round, soft(M_i - U^(T-1) V_i^T), rebuilt by the S-pass
      // tile code itself so that it is bitwise the S the round used.
      // The kernel indexes S by global column; shift the base so that client
      // b's first column lands at S. Only clients [b, e) are launched.
      float* base = S - c->col_off[b] * lds;
      RPCA_HIP(c, launch_spass(q, c->U[c->cur ^ 1], 0, base, lds, 1, b, e - b, c->stream),
               "S emit launch");
    }
  }
  return RPCA_OK;
}

rpca_status rpca_get_factors(rpca_ctx* c, float* U, int64_t ldu, float* V, int64_t ldv) {
  if (rpca_status s = guard(c)) return s;
  if ((U && ldu < c->p.m) || (V && ldv < c->p.n)) return fail(c, RPCA_EINVAL, "leading dimension too small");
  RPCA_HIP(c,
           launch_get_factors(with_v(c, c->vcur), c->clients.data(), c->col_off.data(), c->U[c->cur], U, ldu, V,
                              ldv, c->stream),
           "factor copy launch");
  return RPCA_OK;
}

rpca_status rpca_get_stats(rpca_ctx* c, int64_t round, rpca_stats* out) {
  if (rpca_status s = guard(c)) return s;
  if (!out) return fail(c, RPCA_EINVAL, "out is NULL");
  if (rpca_status s = flush_finalize(c)) return s;
  if (round < 0) round = c->rounds - 1;
  if (round < 0 || round >= c->rounds || round < c->rounds - kHist)
    return fail(c, RPCA_EINVAL, "round not available");
  StatsRec rec;
  RPCA_HIP(c,
           hipMemcpyAsync(&rec, c->p.hist + round % kHist, sizeof(rec), hipMemcpyDeviceToHost,
                          c->stream),
           "copy stats");
  RPCA_HIP(c, hipStreamSynchronize(c->stream), "synchronize");
  std::memcpy(out, &rec, sizeof(rec));
  return RPCA_OK;
}

rpca_status rpca_profile(rpca_ctx* c, int32_t rounds, double* avg_ms, int64_t* launches) {
  if (rpca_status s = guard(c)) return s;
  if (rounds < 1 || !avg_ms || !launches) return fail(c, RPCA_EINVAL, "bad profile arguments");
  Profiler prof;
  for (int32_t t = 0; t < rounds; ++t)
    if (rpca_status s = enqueue_round(c, &prof)) return s;
  RPCA_HIP(c, hipStreamSynchronize(c->stream), "synchronize");
  double tot[RPCA_NUM_PHASES] = {0};
  int64_t cnt[RPCA_NUM_PHASES] = {0};
  for (size_t k = 0; k < prof.phase.size(); ++k) {
    float ms = 0.f;
    RPCA_HIP(c, hipEventElapsedTime(&ms, prof.ev[2 * k], prof.ev[2 * k + 1]), "elapsed time");
    tot[prof.phase[k]] += ms;
    cnt[prof.phase[k]] += 1;
  }
  for (int k = 0; k < RPCA_NUM_PHASES; ++k) {
    avg_ms[k] = cnt[k] ? tot[k] / (double)cnt[k] : 0.0;
    launches[k] = cnt[k];
  }
  return RPCA_OK;
}

int64_t rpca_rounds(const rpca_ctx* c) { return c ? c->rounds : -1; }

const char* rpca_last_error(const rpca_ctx* c) {
  if (!c) return g_init_err.c_str();
  return c->err.c_str();
}

void rpca_destroy(rpca_ctx* c) {
  if (!c) return;
  if (c->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
  }
  for (hipGraphExec_t& g : c->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  delete c;
}

}  // extern "C"
