// TRPL+K driver and C ABI.
//
// The host sequences kernel launches on the context stream; all n-length
// work runs on the device.  Per restart cycle the host reads back one small
// report (the Ritz values and residual norms of the kept Ritz pairs, O(m)
// doubles) to take the locking and target decisions of Alg. 1; everything
// inside a cycle is launched without a host synchronisation.  The basis size
// lives in device memory (DevState::nb) so that an invariant-subspace
// breakdown or a dropped +K vector detected on the device turns the rest of
// the stage into no-ops.
//
// Memory layout (all float64, column-major, leading dimension ld = n rounded
// up to 32 elements, i.e. 256-byte aligned columns):
//   W  = [Q | U]   locked vectors (hard locking) followed by the active
//                  basis; locking a converged Ritz vector only moves the start
//                  u0 of U one column to the right, so [Q, U] stays one
//                  contiguous block for the Gram-Schmidt passes.
//   AW = A W, BW = B W (BW only for B != I).
//   T (m x m), theta (m), Y (m x m), the previous Ritz vectors (n x l) and
//   a handful of n-vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/trplk.h"
#include "common.h"

using namespace trplk;

namespace {

constexpr double BREAKDOWN_TOL = 1e-14;  // inner-step breakdown (relative)
constexpr int MIXED_STALL_CYCLES = 8;    // float32 phase: cycles without halving the residual
constexpr double PLUSK_DROP_TOL = 1e-12; // +K vector dropped when nearly dependent
constexpr int BLOCK_MAX = 16;            // largest inner block of block TRPL+K

struct DevCsr {
  int n = 0;
  int64_t nnz = 0;
  int* rowptr = nullptr;
  int* col = nullptr;
  double* val = nullptr;
  float* val32 = nullptr;
  bool owned = false;
  SpmvPlan plan;
};

// start blocks of at least this many vectors are orthonormalised by Cholesky
// QR on the matrix cores (fewer: column by column)
constexpr int CHOLQR_MIN_K = 8;
constexpr int START_BY_COLUMNS = 100;  // start_cholqr: fall back to the column-by-column start

struct Report {
  int nb;
  int bad;
  int pl1_err;
  int pad;
  long long cnt_append;
  long long cnt_norm;
  double theta[SYEV_MAXB];
  double res[SYEV_MAXB];
  double xn[SYEV_MAXB];
};

struct Prof {
  hipEvent_t a, b;
  int cls;
  int64_t bytes;
};

}  // namespace

struct trplk_ctx {
  hipStream_t s = nullptr;
  trplk_opts o{};
  int n = 0;
  DevCsr A, B;
  bool hasB = false;
  int prec = TRPLK_PREC_NONE;
  double* dinv = nullptr;
  DevCsr G, Gt;  // factor preconditioner M = G^T G
  double normA_inf = 0.0, normA_fro = 0.0;
  // workspace
  int64_t ld = 0;
  int pcap = 0;  // locked-vector capacity
  int m = 0;
  double* W = nullptr;
  double* AW = nullptr;
  double* BW = nullptr;
  double* w = nullptr;
  double* wtmp = nullptr;
  double* tmpB = nullptr;
  double* vtmp = nullptr;
  double* ytmp = nullptr;
  float* v32 = nullptr;
  float* y32 = nullptr;
  float* wtmp32 = nullptr;
  double* Xprev = nullptr;
  double* pl1_Ap = nullptr;  // PL+1: A p and B p of the search direction (p itself in Xprev)
  double* pl1_Bp = nullptr;
  double* pl1_s = nullptr;   // PL+1: border of Q^T B Q (2 * ORTH_MAXCOL)
  double* pl1_work = nullptr;  // PL+1: the projected pencil's matrices (pl1_work_doubles())
  int* pl1_q = nullptr;        // PL+1: columns of the pencil used, p_{k-1} kept
  int* cq_flag = nullptr;      // start block by Cholesky QR: 1 = the Gram matrix was too close to singular
  double* T = nullptr;
  double* theta = nullptr;
  double* Y = nullptr;
  double* hbuf = nullptr;
  double* cbuf = nullptr;   // delayed form: correction coefficients of the pending column
  double* Lm = nullptr;     // delayed form: AU_true = AU_stored Lm (SYEV_MAXB^2)
  double* YA = nullptr;     // delayed form: Lm Y, the rotation coefficients of AU
  double* partial = nullptr;
  double* resout = nullptr;
  double* thout = nullptr;  // Ritz values of the returned pairs (get_eigpairs)
  // block TRPL+K (opts.block > 1): the current inner block, reduction
  // partials of the block passes, coefficients, small scalars, target shifts
  double* Wblk = nullptr;
  double* bpart = nullptr;
  double* bh = nullptr;
  double* bsmall = nullptr;
  double* bshift = nullptr;
  DevState* st = nullptr;
  Report* rep_h = nullptr;
  Report* rep_d = nullptr;
  int orth_nblk = 0, rot_nblk = 0;  // orth_nblk: largest pass grid (sizes partials)
  int64_t partial_bytes = 0;
  int64_t partial_cap = 0;  // doubles in `partial`
  bool ws_ready = false;
  void* ws_base = nullptr;  // caller's workspace (trplk_create_ws), not owned
  int64_t ws_size = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> evpool;
  std::vector<Prof> prof;
  size_t evused = 0;
  // results
  bool solved = false;
  int u0 = 0;             // locked columns in front of U
  int nout = 0;           // result columns in W starting at column 0
  std::vector<double> theta_out, res_out;
  std::vector<int> conv_out;
  std::vector<double> hist;  // smallest active Ritz value after each cycle's Rayleigh-Ritz
  trplk_stats stats{};
  std::string err;
  int64_t dev_bytes = 0;
  bool fp32_phase = false;
  // learned factor: pattern of tril(A), its transpose, features, parameters
  // and the training buffers (built on first use)
  struct Learn {
    bool ready = false;
    bool pairs = false;
    int S = 0;
    int pair_cap = 0;   // pairs the pair buffers hold
    int64_t nnz = 0;
    int* Lrow = nullptr;
    int* Lcol = nullptr;
    int* lr = nullptr;
    double* lval = nullptr;
    int* Trow = nullptr;
    int* Tcol = nullptr;
    double* permd = nullptr;
    double* dinv = nullptr;
    double* F = nullptr;
    float* Fz = nullptr;
    double* gval = nullptr;
    double* gvalT = nullptr;
    float* P = nullptr;
    float* am = nullptr;
    float* av = nullptr;
    double* Er = nullptr;
    double* Rr = nullptr;
    double* Y = nullptr;
    double* D = nullptr;
    double* Uu = nullptr;
    double* Z = nullptr;
    double* coef = nullptr;
    double* w = nullptr;
    float* dout = nullptr;
    double* part = nullptr;
    double* loss = nullptr;
    double* grad = nullptr;
    double* scratch = nullptr;
    double* cbar = nullptr;
  } L;
};

static std::string g_create_err;

namespace {

int set_err(trplk_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_err(ctx, TRPLK_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t dalloc(trplk_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e == hipSuccess) c->dev_bytes += static_cast<int64_t>(count * sizeof(T));
  return e;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

int validate_host_csr(const trplk_csr* M, int n, std::string& why) {
  if (!M || !M->rowptr || !M->col || !M->val) {
    why = "null CSR array";
    return TRPLK_EINVAL;
  }
  if (M->n != n || M->n < 1) {
    why = "CSR dimension mismatch";
    return TRPLK_EINVAL;
  }
  if (M->nnz < 0 || M->nnz >= (int64_t(1) << 31)) {
    why = "nnz out of range";
    return TRPLK_EINVAL;
  }
  if (M->rowptr[0] != 0 || M->rowptr[n] != M->nnz) {
    why = "rowptr[0] must be 0 and rowptr[n] must equal nnz";
    return TRPLK_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    if (M->rowptr[i + 1] < M->rowptr[i]) {
      why = "rowptr not monotone";
      return TRPLK_EINVAL;
    }
    for (int j = M->rowptr[i]; j < M->rowptr[i + 1]; ++j) {
      if (M->col[j] < 0 || M->col[j] >= n) {
        why = "column index out of range";
        return TRPLK_EINVAL;
      }
      if (j > M->rowptr[i] && M->col[j] <= M->col[j - 1]) {
        why = "columns not sorted or duplicated";
        return TRPLK_EINVAL;
      }
      if (!std::isfinite(M->val[j])) {
        why = "non-finite matrix value";
        return TRPLK_ENUMERIC;
      }
    }
  }
  return TRPLK_OK;
}

int64_t dia_bytes(const SpmvPlan& p) {
  return static_cast<int64_t>(p.ndiag) * p.n * ((p.dia_val ? 8 : 0) + (p.dia_val32 ? 4 : 0));
}

int upload_csr(trplk_ctx* c, DevCsr& D, const trplk_csr* M, int32_t mem, bool want32) {
  D.n = M->n;
  D.nnz = M->nnz;
  if (mem == TRPLK_MEM_HOST) {
    D.owned = true;
    HIPCHK(c, dalloc(c, &D.rowptr, D.n + 1));
    HIPCHK(c, dalloc(c, &D.col, std::max<int64_t>(D.nnz, 1)));
    HIPCHK(c, dalloc(c, &D.val, std::max<int64_t>(D.nnz, 1)));
    HIPCHK(c, hipMemcpyAsync(D.rowptr, M->rowptr, sizeof(int) * (D.n + 1), hipMemcpyHostToDevice, c->s));
    HIPCHK(c, hipMemcpyAsync(D.col, M->col, sizeof(int) * D.nnz, hipMemcpyHostToDevice, c->s));
    HIPCHK(c, hipMemcpyAsync(D.val, M->val, sizeof(double) * D.nnz, hipMemcpyHostToDevice, c->s));
  } else {
    D.owned = false;
    D.rowptr = const_cast<int*>(M->rowptr);
    D.col = const_cast<int*>(M->col);
    D.val = const_cast<double*>(M->val);
  }
  if (want32) {
    HIPCHK(c, dalloc(c, &D.val32, std::max<int64_t>(D.nnz, 1)));
    HIPCHK(c, cast_f32(D.nnz, D.val, D.val32, c->s));
  }
  HIPCHK(c, spmv_plan(D.plan, D.n, D.rowptr, 0, c->s));
  HIPCHK(c, spmv_plan_dia(D.plan, D.n, D.rowptr, D.col, D.val, D.val32, c->s));
  c->dev_bytes += dia_bytes(D.plan);
  return TRPLK_OK;
}

void free_csr(DevCsr& D) {
  if (D.owned) {
    dfree(D.rowptr);
    dfree(D.col);
    dfree(D.val);
  }
  dfree(D.val32);
  spmv_plan_free(D.plan);
  D = DevCsr();
}

// ------------------------------------------------------------ profiling --
enum { PC_SPMV = 0, PC_ORTH = 1, PC_PREC = 2, PC_ROT = 3, PC_RR = 4, PC_DOT = 5, PC_UPDDOT = 6,
       PC_UPD = 7, PC_DCDOT = 8, PC_DCUPD = 9 };

struct ProfScope {
  trplk_ctx* c;
  size_t idx = SIZE_MAX;
  ProfScope(trplk_ctx* ctx, int cls, int64_t bytes) : c(ctx) {
    if (!c->o.profile) return;
    if (c->evused + 2 > c->evpool.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->evpool.push_back(e);
      }
    }
    Prof p{c->evpool[c->evused], c->evpool[c->evused + 1], cls, bytes};
    c->evused += 2;
    (void)hipEventRecord(p.a, c->s);
    idx = c->prof.size();
    c->prof.push_back(p);
  }
  ~ProfScope() {
    if (idx != SIZE_MAX) (void)hipEventRecord(c->prof[idx].b, c->s);
  }
};

// ------------------------------------------------------------ workspace --
// The n-length part of the solver workspace: W = [Q | U], A W, B W, the
// previous Ritz vectors, PL+1's search-direction products and the n-vectors.
// It is carved in this order from one region (256-byte aligned pieces): the
// caller's workspace (trplk_create_ws) or one allocation per piece.
struct WsPiece {
  void** ptr;
  int64_t bytes;
};

bool hard_locking(const trplk_opts& o) {
  return (o.locking == TRPLK_LOCK_HARD) || (o.locking == TRPLK_LOCK_AUTO && o.p > o.k);
}

int64_t ws_align(int64_t b) { return (b + 255) / 256 * 256; }

void ws_pieces(trplk_ctx* c, std::vector<WsPiece>& out) {
  const trplk_opts& o = c->o;
  const int64_t ld = (static_cast<int64_t>(c->n) + 31) / 32 * 32;
  const int64_t cols = (hard_locking(o) ? o.p : 0) + o.m;
  const int64_t d = 8 * ld, f = 4 * ld;
  out.clear();
  out.push_back({reinterpret_cast<void**>(&c->W), d * cols});
  out.push_back({reinterpret_cast<void**>(&c->AW), d * cols});
  if (c->hasB) out.push_back({reinterpret_cast<void**>(&c->BW), d * cols});
  out.push_back({reinterpret_cast<void**>(&c->Xprev), d * std::max(o.l, 1)});
  out.push_back({reinterpret_cast<void**>(&c->pl1_Ap), d});
  if (c->hasB) out.push_back({reinterpret_cast<void**>(&c->pl1_Bp), d});
  out.push_back({reinterpret_cast<void**>(&c->w), d});
  out.push_back({reinterpret_cast<void**>(&c->wtmp), d});
  out.push_back({reinterpret_cast<void**>(&c->vtmp), d});
  out.push_back({reinterpret_cast<void**>(&c->ytmp), d});
  if (c->hasB) out.push_back({reinterpret_cast<void**>(&c->tmpB), d});
  out.push_back({reinterpret_cast<void**>(&c->v32), f});
  out.push_back({reinterpret_cast<void**>(&c->y32), f});
  out.push_back({reinterpret_cast<void**>(&c->wtmp32), f});
  if (o.block > 1) out.push_back({reinterpret_cast<void**>(&c->Wblk), d * o.block});
}

int64_t ws_bytes_needed(trplk_ctx* c) {
  std::vector<WsPiece> pcs;
  ws_pieces(c, pcs);
  int64_t b = 0;
  for (const WsPiece& q : pcs) b += ws_align(q.bytes);
  return b;
}

int ensure_workspace(trplk_ctx* c) {
  if (c->ws_ready) return TRPLK_OK;
  const int n = c->n;
  const trplk_opts& o = c->o;
  c->m = o.m;
  c->ld = (static_cast<int64_t>(n) + 31) / 32 * 32;
  c->pcap = hard_locking(o) ? o.p : 0;
  std::vector<WsPiece> pcs;
  ws_pieces(c, pcs);
  if (c->ws_base) {
    const int64_t need = ws_bytes_needed(c);
    if (c->ws_size < need)
      return set_err(c, TRPLK_EINVAL, "workspace smaller than trplk_workspace_size()");
    char* base = static_cast<char*>(c->ws_base);
    int64_t off = 0;
    for (const WsPiece& q : pcs) {
      *q.ptr = base + off;
      off += ws_align(q.bytes);
    }
  } else {
    for (const WsPiece& q : pcs) {
      char* ptr = nullptr;
      HIPCHK(c, dalloc(c, &ptr, static_cast<size_t>(q.bytes)));
      *q.ptr = ptr;
    }
  }
  HIPCHK(c, dalloc(c, &c->T, SYEV_MAXB * SYEV_MAXB));
  HIPCHK(c, dalloc(c, &c->theta, SYEV_MAXB));
  HIPCHK(c, dalloc(c, &c->Y, SYEV_MAXB * SYEV_MAXB));
  HIPCHK(c, dalloc(c, &c->hbuf, ORTH_MAXCOL));
  HIPCHK(c, dalloc(c, &c->cbuf, ORTH_MAXCOL));
  HIPCHK(c, dalloc(c, &c->Lm, SYEV_MAXB * SYEV_MAXB));
  HIPCHK(c, dalloc(c, &c->YA, SYEV_MAXB * SYEV_MAXB));
  HIPCHK(c, dalloc(c, &c->resout, 2 * SYEV_MAXB));
  HIPCHK(c, dalloc(c, &c->thout, SYEV_MAXB));
  HIPCHK(c, dalloc(c, &c->pl1_s, 2 * ORTH_MAXCOL));
  if (o.method != TRPLK_METHOD_TRPLK) {
    HIPCHK(c, dalloc(c, &c->pl1_work, static_cast<size_t>(pl1_work_doubles())));
    HIPCHK(c, dalloc(c, &c->pl1_q, 2));
  }
  if (o.block > 1 || (o.method == TRPLK_METHOD_TRPLK && o.k >= CHOLQR_MIN_K))
    HIPCHK(c, dalloc(c, &c->bpart, static_cast<size_t>(block_partial_doubles())));
  HIPCHK(c, dalloc(c, &c->cq_flag, 1));
  if (o.block > 1) {
    HIPCHK(c, dalloc(c, &c->bh, ORTH_MAXCOL * BLOCK_MAX));
    HIPCHK(c, dalloc(c, &c->bsmall, 4 * BLOCK_MAX));
    HIPCHK(c, dalloc(c, &c->bshift, BLOCK_MAX));
  }
  c->orth_nblk = orth_blocks_max(n);
  c->rot_nblk = rot_blocks(n);
  int64_t pb = static_cast<int64_t>(c->orth_nblk) * orth_stride();
  pb = std::max<int64_t>(pb, static_cast<int64_t>(c->rot_nblk) * 128);
  pb = std::max<int64_t>(pb, spmv_partial_blocks(c->A.plan));
  if (c->hasB) pb = std::max<int64_t>(pb, spmv_partial_blocks(c->B.plan));
  pb = std::max<int64_t>(pb, 2 * static_cast<int64_t>(rownorm_blocks(n)));
  HIPCHK(c, dalloc(c, &c->partial, pb));
  c->partial_cap = pb;
  HIPCHK(c, dalloc(c, &c->st, 1));
  HIPCHK(c, hipMemsetAsync(c->st, 0, sizeof(DevState), c->s));
  HIPCHK(c, hipHostMalloc(reinterpret_cast<void**>(&c->rep_h), sizeof(Report)));
  HIPCHK(c, dalloc(c, &c->rep_d, 1));
  HIPCHK(c, hipEventCreate(&c->ev0));
  HIPCHK(c, hipEventCreate(&c->ev1));
  c->ws_ready = true;
  return TRPLK_OK;
}

// ---------------------------------------------------------- start block --
// The default start block is uniform on [-1, 1) (the paper starts from a
// seeded random block, Sec. 5).  Entry e of the column-major n x k block is
// the e-th output of SplitMix64 (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) seeded with `seed`: the
// state seed + (e + 1) * gamma, gamma = 0x9e3779b97f4a7c15, through the
// generator's 64-bit finaliser; its top 53 bits b give b * 2^-52 - 1.  The
// scaling is exact and the subtraction rounds once, so any IEEE
// implementation of the same definition produces the same doubles.
__device__ __forceinline__ uint64_t splitmix64_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_start_column(int n, uint64_t seed, uint64_t first, double* w) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t e = first + static_cast<uint64_t>(i);
    const uint64_t z = splitmix64_out(seed + (e + 1ull) * 0x9e3779b97f4a7c15ull);
    w[i] = static_cast<double>(z >> 11) * 0x1.0p-52 - 1.0;
  }
}

// ------------------------------------------------------------- building --
// The report kernel copies the device scalars the host needs once per cycle.
__global__ void k_report(const DevState* st, const double* theta, const double* resout, int nth,
                         int nres, Report* rep) {
  const int t = threadIdx.x;
  if (t == 0) {
    rep->nb = st->nb;
    rep->bad = st->bad;
    rep->pl1_err = st->pl1_err;
    rep->cnt_append = st->cnt_append;
    rep->cnt_norm = st->cnt_norm;
  }
  if (t < nth && t < SYEV_MAXB) rep->theta[t] = theta[t];
  if (t < nres && t < SYEV_MAXB) {
    rep->res[t] = resout[t];
    rep->xn[t] = resout[64 + t];
  }
}

struct Solver {
  trplk_ctx* c;
  int n;
  int64_t ld;
  hipStream_t s;
  int nbh = 0;  // host-side expected basis size
  bool keepT = false;  // the next cycle keeps T(0:kact,0:kact) (recomputed X^T A X)
  int skip0 = 0;  // PL+1: inner vectors are not orthogonalised against the first column
  bool dc = false;  // delayed re-orthogonalisation of the inner vectors

  double* Ucol(int j) const { return c->W + (c->u0 + j) * ld; }
  double* AUcol(int j) const { return c->AW + (c->u0 + j) * ld; }
  double* BUcol(int j) const { return c->hasB ? c->BW + (c->u0 + j) * ld : Ucol(j); }
  double* Wq() const { return c->W; }              // [Q | U] start
  double* BWq() const { return c->hasB ? c->BW : c->W; }

  // matrix (in the format launched) + x read + y written
  int64_t spmv_bytes(const DevCsr& M, bool f32) const {
    const int64_t vb = f32 ? 4 : 8;
    return spmv_matrix_bytes(M.plan, M.nnz, f32) + 2 * vb * M.n;
  }

  hipError_t orth(int mode, const OrthArgs& a) {
    int64_t cols = a.ncol_fixed + a.ncol_extra + (a.state ? nbh : 0);
    int64_t bytes;
    const bool same = (mode == ORTH_DOT) ? (a.nvec == 1 || a.Md0 == a.Md1) : (a.Mu == a.Md1);
    if (mode == ORTH_DOT) bytes = 8 * cols * n * (same ? 1 : 2) + 8LL * n * a.nvec;
    else if (mode == ORTH_UPD_DOT) bytes = 8 * cols * n * (same ? 1 : 2) + 16LL * n;
    else if (mode == ORTH_UPD2) {
      const bool gen = a.Md1 && a.Md1 != a.Mu;  // B U corrected as well
      bytes = 8 * (cols - 1) * n * (gen ? 2 : 1) + (gen ? 32LL : 16LL) * n + (a.w ? 16LL : 0LL) * n;
    }
    else bytes = 8 * cols * n + 16LL * n;
    const int cls = mode == ORTH_DOT ? (a.nvec == 3 ? PC_DCDOT : PC_DOT)
                    : mode == ORTH_UPD_DOT ? PC_UPDDOT : mode == ORTH_UPD2 ? PC_DCUPD : PC_UPD;
    ProfScope ps(c, cls, bytes);
    const int g = (mode == ORTH_DOT && a.nvec == 3) ? orth_blocks_dot3(n) : orth_blocks(n, mode);
    // every block writes one row of partials
    if (static_cast<int64_t>(g) * orth_stride() > c->partial_cap) return hipErrorInvalidValue;
    return orth_pass(mode, a, g, s);
  }
  int nblk(int mode) const { return orth_blocks(n, mode); }

  hipError_t spmv(const DevCsr& M, const SpmvArgs& a, bool f32, int cls, int64_t extra_bytes) {
    ProfScope ps(c, cls, spmv_bytes(M, f32) + extra_bytes);
    return f32 ? spmv_f32(M.plan, a, s) : spmv_f64(M.plan, a, s);
  }

  hipError_t fin(const FinishArgs& f) { return finish(f, s); }

  int maxcols() const { return c->u0 + c->m + 1; }

  // B-CGS2 of the vector in c->w against [Q | U(:, 0:nb)]; leaves the
  // projected vector in c->wtmp (and wtmp32), its B-norm in the state.
  // first_pass: false when h1 is already in hbuf (fused with the T column).
  int project(bool first_pass) {
    Status S;
    const int ncf = c->u0;
    if (first_pass) {
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = ncf; a.state = c->st; a.ncol_max = maxcols();
      a.Md0 = BWq(); a.vec0 = c->w; a.nvec = 1; a.partial = c->partial;
      S.check(orth(ORTH_DOT, a), "orth h1");
      FinishArgs f;
      f.mode = FIN_H; f.partial = c->partial; f.nblk = nblk(ORTH_DOT); f.stride = orth_stride();
      f.state = c->st; f.ncol_fixed = ncf; f.h = c->hbuf; f.skip_first = skip0;
      S.check(fin(f), "fin h1");
    }
    {
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = ncf; a.state = c->st; a.ncol_max = maxcols();
      a.Mu = Wq(); a.Md1 = BWq(); a.h = c->hbuf; a.w = c->w; a.partial = c->partial;
      S.check(orth(ORTH_UPD_DOT, a), "orth upd-dot");
      FinishArgs f;
      f.mode = FIN_H2; f.partial = c->partial; f.nblk = nblk(ORTH_UPD_DOT); f.stride = orth_stride();
      f.state = c->st; f.ncol_fixed = ncf; f.h = c->hbuf; f.skip_first = skip0;
      S.check(fin(f), "fin h2");
    }
    {
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = ncf; a.state = c->st; a.ncol_max = maxcols();
      a.Mu = Wq(); a.h = c->hbuf; a.w = c->w; a.wout = c->wtmp;
      a.wout32 = c->fp32_phase ? c->wtmp32 : nullptr;
      a.norm = !c->hasB; a.partial = c->partial;
      a.fuse_norm = a.norm;  // B = I: the pass's last workgroup takes the decision
      S.check(orth(ORTH_UPD, a), "orth upd");
    }
    if (c->hasB) {
      FinishArgs f;
      f.mode = FIN_NORM; f.state = c->st; f.partial = c->partial;
      SpmvArgs b;
      b.n = n; b.rowptr = c->B.rowptr; b.col = c->B.col; b.val = c->B.val; b.x = c->wtmp;
      b.mode = SPMV_DOT; b.state = c->st; b.y = c->tmpB; b.xd = c->wtmp; b.partial = c->partial;
      S.check(spmv(c->B, b, false, PC_SPMV, 8LL * n), "spmv B");
      f.nblk = spmv_partial_blocks(c->B.plan);
      f.stride = 1;
      S.check(fin(f), "fin norm");
    }
    return S.ok() ? TRPLK_OK : set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
  }

  // Append wtmp / beta as basis column nb; z = A g into AU.  next selects the
  // formation of the next inner direction in the epilogue.
  int append(int next) {
    Status S;
    SpmvArgs a;
    const bool f32 = c->fp32_phase;
    a.n = n; a.rowptr = c->A.rowptr; a.col = c->A.col;
    a.val = f32 ? static_cast<const void*>(c->A.val32) : static_cast<const void*>(c->A.val);
    a.x = f32 ? static_cast<const void*>(c->wtmp32) : static_cast<const void*>(c->wtmp);
    a.mode = SPMV_APPEND; a.use_beta = true; a.state = c->st; a.xd = c->wtmp;
    a.bx = c->hasB ? c->tmpB : nullptr;
    a.U = c->W; a.AU = c->AW; a.BU = c->BW; a.ld = ld; a.col0 = c->u0;
    int64_t extra = 8LL * n * (c->hasB ? 4 : 2);
    if (next == 1) {
      if (c->prec == TRPLK_PREC_JACOBI) {
        a.next = NEXT_JACOBI; a.dinv = c->dinv; a.wout = c->w; extra += 16LL * n;
      } else if (c->prec == TRPLK_PREC_NONE) {
        a.next = NEXT_IDENT; a.wout = c->w; extra += 8LL * n;
      } else {
        a.next = NEXT_STORE_V;
        if (c->o.precision == TRPLK_MIXED) { a.vout32 = c->v32; extra += 4LL * n; }
        else { a.vout = c->vtmp; extra += 8LL * n; }
      }
    }
    S.check(spmv(c->A, a, f32, PC_SPMV, extra), "spmv append");
    if (next == 1 && c->prec >= TRPLK_PREC_FSAI) S.check(apply_factor(), "factor");
    return S.ok() ? TRPLK_OK : set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
  }

  // w = G^T (G v) with v in vtmp (float64) or v32 (mixed)
  hipError_t apply_factor() {
    const bool f32 = c->o.precision == TRPLK_MIXED;
    SpmvArgs a;
    a.n = n; a.rowptr = c->G.rowptr; a.col = c->G.col; a.state = c->st; a.mode = SPMV_STORE;
    a.val = f32 ? static_cast<const void*>(c->G.val32) : static_cast<const void*>(c->G.val);
    a.x = f32 ? static_cast<const void*>(c->v32) : static_cast<const void*>(c->vtmp);
    a.y = f32 ? static_cast<void*>(c->y32) : static_cast<void*>(c->ytmp);
    hipError_t e = spmv(c->G, a, f32, PC_PREC, 0);
    if (e != hipSuccess) return e;
    SpmvArgs b;
    b.n = n; b.rowptr = c->Gt.rowptr; b.col = c->Gt.col; b.state = c->st; b.mode = SPMV_STORE;
    b.val = f32 ? static_cast<const void*>(c->Gt.val32) : static_cast<const void*>(c->Gt.val);
    b.x = f32 ? static_cast<const void*>(c->y32) : static_cast<const void*>(c->ytmp);
    b.y = c->w; b.out_f64 = true;
    return spmv(c->Gt, b, f32, PC_PREC, f32 ? 4LL * n : 0);
  }

  // T column of the vector just appended: T(0:nb, nb) = U^T z (after
  // increments nb), optionally fused with h1 = BW^T w for the next direction.
  int tcol(bool with_h1) {
    Status S;
    OrthArgs a;
    a.n = n; a.ld = ld; a.ncol_fixed = c->u0; a.ncol_extra = 1; a.state = c->st;
    a.ncol_max = maxcols();
    a.Md0 = Wq(); a.vec0_base = c->AW; a.vec0_col0 = c->u0; a.partial = c->partial;
    if (with_h1) {
      a.nvec = 2; a.Md1 = BWq(); a.vec1 = c->w;
    } else {
      a.nvec = 1;
    }
    S.check(orth(ORTH_DOT, a), "orth tcol");
    FinishArgs f;
    f.mode = with_h1 ? FIN_TH : FIN_T; f.partial = c->partial; f.nblk = nblk(ORTH_DOT);
    f.stride = orth_stride(); f.state = c->st; f.ncol_fixed = c->u0; f.T = c->T; f.ldT = SYEV_MAXB;
    f.h = c->hbuf; f.skip_first = skip0;
    S.check(fin(f), "fin tcol");
    return S.ok() ? TRPLK_OK : set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
  }

  // Delayed form, first inner vector: one Gram-Schmidt pass of w against
  // [Q | U] into wtmp with its norm; the second pass is merged into the
  // next dc_step.
  // Norm of the once-orthogonalised vector in wtmp and its acceptance test
  // (delayed form).  For B = I the update pass left ||wtmp||^2 partials and
  // its last workgroup took the decision (fuse_norm); for B != I one product
  // B wtmp (kept in tmpB for the append) gives the B-norm.
  void norm_finish(Status& S) {
    if (!c->hasB) return;
    FinishArgs f;
    f.mode = FIN_NORM; f.state = c->st; f.partial = c->partial; f.dc = 1;
    SpmvArgs b;
    b.n = n; b.rowptr = c->B.rowptr; b.col = c->B.col; b.val = c->B.val; b.x = c->wtmp;
    b.mode = SPMV_DOT; b.state = c->st; b.y = c->tmpB; b.xd = c->wtmp; b.partial = c->partial;
    S.check(spmv(c->B, b, false, PC_SPMV, 8LL * n), "spmv B");
    f.nblk = spmv_partial_blocks(c->B.plan);
    f.stride = 1;
    S.check(fin(f), "fin norm");
  }

  int project_once() {
    Status S;
    const int ncf = c->u0;
    {
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = ncf; a.state = c->st; a.ncol_max = maxcols();
      a.Md0 = BWq(); a.vec0 = c->w; a.nvec = 1; a.partial = c->partial;
      S.check(orth(ORTH_DOT, a), "orth h");
      FinishArgs f;
      f.mode = FIN_H; f.partial = c->partial; f.nblk = nblk(ORTH_DOT); f.stride = orth_stride();
      f.state = c->st; f.ncol_fixed = ncf; f.h = c->hbuf;
      S.check(fin(f), "fin h");
    }
    {
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = ncf; a.state = c->st; a.ncol_max = maxcols();
      a.Mu = Wq(); a.h = c->hbuf; a.w = c->w; a.wout = c->wtmp;
      a.wout32 = c->fp32_phase ? c->wtmp32 : nullptr;
      a.norm = !c->hasB; a.partial = c->partial;
      a.fuse_norm = a.norm; a.norm_dc = 1;
      S.check(orth(ORTH_UPD, a), "orth upd");
    }
    norm_finish(S);
    return S.ok() ? TRPLK_OK : set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
  }

  // Delayed form, after the append of u' (column nb, once orthogonalised)
  // with z' = A u', B u' and, when `more`, the next direction
  // w = M(z' - rho B u'): one dot pass gives U^T B u', U^T z' and (B U)^T w;
  // the finish kernel turns them into the correction c, the exact T column
  // of the corrected vector and the coefficients of w; one update pass
  // writes u = (u' - U c) / gamma (and B u) in place and the
  // once-orthogonalised w into wtmp, whose (B-)norm follows.
  // plusk: the vector in c->w is a +K vector; the column at nb is corrected
  // only if it is pending (not after a breakdown of the Krylov block)
  int dc_step(bool more, bool plusk = false) {
    Status S;
    const int ncf = c->u0;
    {
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = ncf; a.ncol_extra = 1; a.state = c->st;
      a.ncol_max = maxcols();
      a.Md0 = Wq(); a.Md1 = BWq(); a.vec0_base = c->hasB ? c->BW : c->W; a.vec1_base = c->AW;
      a.vec0_col0 = ncf;
      // three vectors also for the last column (the third, w, is then unused):
      // the finish reads the packed three-vector layout
      a.nvec = 3; a.vec2 = c->w; a.partial = c->partial;
      S.check(orth(ORTH_DOT, a), "orth dc dot");
      FinishArgs f;
      f.mode = FIN_DC; f.partial = c->partial; f.nblk = orth_blocks_dot3(n); f.stride = orth_stride();
      f.state = c->st; f.ncol_fixed = ncf; f.T = c->T; f.ldT = SYEV_MAXB; f.h = c->hbuf;
      f.nvec = more ? 3 : 2; f.cbuf = c->cbuf; f.L = c->Lm; f.dc = plusk ? 1 : 0;
      f.cnt = 3 * maxcols();  // bound on the packed row width 3 (J + 1)
      S.check(fin(f), "fin dc");
    }
    {
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = ncf; a.ncol_extra = 1; a.state = c->st;
      a.ncol_max = maxcols();
      a.Mu = Wq(); a.Md1 = c->hasB ? BWq() : nullptr; a.c = c->cbuf; a.h = c->hbuf;
      a.partial = c->partial;
      if (more) {
        a.w = c->w; a.wout = c->wtmp; a.wout32 = c->fp32_phase ? c->wtmp32 : nullptr;
        a.norm = !c->hasB;
        a.fuse_norm = a.norm; a.norm_dc = 1;
      }
      S.check(orth(ORTH_UPD2, a), "orth dc upd");
    }
    if (more) norm_finish(S);
    return S.ok() ? TRPLK_OK : set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
  }

  int stage_reset(double tol) {
    HIPCHK(c, set_state(c->st, SET_RESET_STAGE, tol * tol, 0, s));
    return TRPLK_OK;
  }

  // orthogonalise + append one non-Krylov vector held in c->w (start block
  // column or +K vector) and fill its T column
  int add_vector(double tol) {
    int r;
    if ((r = stage_reset(tol))) return r;
    if ((r = project(true))) return r;
    if ((r = append(0))) return r;
    if ((r = tcol(false))) return r;
    ++nbh;
    return TRPLK_OK;
  }

  // Column j of the start block into w: copied from src, or, when src is
  // NULL, drawn on the device from the seeded counter-based stream.
  int load_w(const double* src, int32_t mem, int j, double* dst = nullptr) {
    if (!dst) dst = c->w;
    if (!src) {
      hipLaunchKernelGGL(k_start_column, dim3(std::max(1, std::min((n + 255) / 256, 4096))), dim3(256), 0, s, n, c->o.seed,
                         static_cast<uint64_t>(j) * static_cast<uint64_t>(n), dst);
      HIPCHK(c, hipGetLastError());
      return TRPLK_OK;
    }
    HIPCHK(c, hipMemcpyAsync(dst, src, sizeof(double) * n,
                             mem == TRPLK_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    return TRPLK_OK;
  }

  // Start block by Cholesky QR applied twice: the k columns are loaded into
  // U (and B U formed), G = U^T B U by the block dot passes, U <- U R^-1
  // (R^T R = G) by the rotation kernel, twice; then A U and T = U^T A U.
  // The span is the start block's, as with column-by-column Gram-Schmidt,
  // and the Rayleigh-Ritz that follows depends only on the span.  Returns
  // START_BY_COLUMNS (state untouched but U) when G is too close to
  // singular: the caller then orthonormalises column by column.
  int start_cholqr(const double* x0, int32_t mem) {
    Status S;
    const int k = c->o.k;
    int r;
    for (int j = 0; j < k; ++j)
      if ((r = load_w(x0 ? x0 + static_cast<int64_t>(j) * n : nullptr, mem, j, Ucol(j)))) return r;
    if (c->hasB) {
      for (int j = 0; j < k; ++j) {
        SpmvArgs b;
        b.n = n; b.rowptr = c->B.rowptr; b.col = c->B.col; b.val = c->B.val; b.x = Ucol(j);
        b.mode = SPMV_STORE; b.y = BUcol(j);
        S.check(spmv(c->B, b, false, PC_SPMV, 0), "start B x");
      }
    }
    for (int pass = 0; pass < 2; ++pass) {
      {
        ProfScope ps(c, PC_ORTH, 8LL * n * k * ((k + 15) / 16 + 1));
        for (int q = 0; q < k; q += 16)
          S.check(block_dot(n, k, Ucol(0), ld, BUcol(q), ld, std::min(16, k - q), c->bpart,
                            c->Lm + static_cast<int64_t>(q) * SYEV_MAXB, SYEV_MAXB, s), "start gram");
      }
      S.check(chol_inv(c->Lm, SYEV_MAXB, k, c->Y, SYEV_MAXB, c->cq_flag, s), "start chol");
      // (the report's pinned pl1_err slot as the landing place; the next
      // report overwrites it)
      S.check(hipMemcpyAsync(&c->rep_h->pl1_err, c->cq_flag, sizeof(int), hipMemcpyDeviceToHost, s), "flag d2h");
      S.check(hipStreamSynchronize(s), "sync start");
      if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
      if (c->rep_h->pl1_err) return START_BY_COLUMNS;
      RotArgs ra;
      ra.n = n; ra.kout = k; ra.b_fixed = k; ra.Y = c->Y; ra.ldY = SYEV_MAXB;
      ra.U = Ucol(0); ra.AU = nullptr; ra.BU = c->hasB ? BUcol(0) : nullptr; ra.ld = ld;
      {
        ProfScope ps(c, PC_ROT, 16LL * n * k * (c->hasB ? 2 : 1));
        S.check(rotate(ra, c->rot_nblk, s), "start rotate");
      }
    }
    // A U (float32 values in the float32 phase, as every other product then)
    const bool f32 = c->fp32_phase;
    for (int j = 0; j < k; ++j) {
      SpmvArgs a;
      a.n = n; a.rowptr = c->A.rowptr; a.col = c->A.col; a.mode = SPMV_STORE; a.y = AUcol(j);
      if (f32) {
        S.check(cast_f32(n, Ucol(j), c->wtmp32, s), "start cast");
        a.val = c->A.val32; a.x = c->wtmp32; a.out_f64 = true;
      } else {
        a.val = c->A.val; a.x = Ucol(j);
      }
      S.check(spmv(c->A, a, f32, PC_SPMV, f32 ? 4LL * n : 0), "start A x");
    }
    {
      ProfScope ps(c, PC_ORTH, 8LL * n * k * ((k + 15) / 16 + 1));
      for (int q = 0; q < k; q += 16)
        S.check(block_dot(n, k, Ucol(0), ld, AUcol(q), ld, std::min(16, k - q), c->bpart,
                          c->T + static_cast<int64_t>(q) * SYEV_MAXB, SYEV_MAXB, s), "start T");
    }
    S.check(symmetrise(c->T, SYEV_MAXB, k, s), "start T sym");
    S.check(start_state(c->st, k, c->hasB, s), "start state");
    if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
    nbh = k;
    return TRPLK_OK;
  }

  // Rayleigh-Ritz on T(0:nb,0:nb), rotation of U, AU, BU to kout columns
  // and residuals of the first `nres` Ritz pairs; fills the host report.
  int rayleigh_ritz(int kout, int nres, bool useL = false) {
    Status S;
    {
      ProfScope ps(c, PC_RR, 0);
      S.check(syev(c->T, SYEV_MAXB, 0, &c->st->nb, 0, c->theta, c->Y, SYEV_MAXB, s), "syev");
      // delayed form: the stored A U columns are z' = A u'; AU_true Y = AU (L Y)
      if (useL) S.check(ly_product(c->Lm, c->Y, c->YA, SYEV_MAXB, c->st, s), "L Y");
    }
    RotArgs r;
    r.n = n; r.kout = kout; r.state = c->st; r.Y = c->Y; r.ldY = SYEV_MAXB; r.b_max = c->m;
    r.YA = useL ? c->YA : nullptr;
    r.U = Ucol(0); r.AU = AUcol(0); r.BU = c->hasB ? BUcol(0) : nullptr; r.ld = ld;
    r.theta = c->theta; r.partial = c->partial;
    {
      const int64_t mats = c->hasB ? 3 : 2;
      ProfScope ps(c, PC_ROT, 8LL * n * (nbh + kout) * mats);
      S.check(rotate(r, c->rot_nblk, s), "rotate");
    }
    FinishArgs f;
    f.mode = FIN_RES; f.partial = c->partial; f.nblk = c->rot_nblk; f.stride = 128;
    f.out = c->resout; f.cnt = nres;
    S.check(fin(f), "fin res");
    hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, s, c->st, c->theta, c->resout, SYEV_MAXB,
                       nres, c->rep_d);
    S.check(hipGetLastError(), "report");
    S.check(hipMemcpyAsync(c->rep_h, c->rep_d, sizeof(Report), hipMemcpyDeviceToHost, s), "d2h");
    S.check(hipStreamSynchronize(s), "sync");
    if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
    const Report& R = *c->rep_h;
    const int kk = std::min(kout, R.nb);
    for (int i = 0; i < kk; ++i)
      if (!std::isfinite(R.theta[i])) return set_err(c, TRPLK_ENUMERIC, "non-finite Ritz value");
    if (R.bad) return set_err(c, TRPLK_ENOTSPD, "B-norm squared not positive or not finite");
    return TRPLK_OK;
  }

  // Recompute A X for the kact active columns in float64 and the projected
  // block T(0:kact, 0:kact) = X^T A X (used when the mixed form switches its
  // SpMV to float64).
  int refresh_products(int kact) {
    Status S;
    for (int j = 0; j < kact; ++j) {
      SpmvArgs a;
      a.n = n; a.rowptr = c->A.rowptr; a.col = c->A.col; a.val = c->A.val; a.x = Ucol(j);
      a.mode = SPMV_STORE; a.y = AUcol(j);
      S.check(spmv(c->A, a, false, PC_SPMV, 0), "refresh spmv");
    }
    for (int j = 0; j < kact; ++j) {
      OrthArgs o;
      o.n = n; o.ld = ld; o.ncol_fixed = j + 1; o.ncol_max = j + 1; o.Md0 = Ucol(0);
      o.vec0 = AUcol(j); o.nvec = 1; o.partial = c->partial;
      S.check(orth(ORTH_DOT, o), "refresh T");
      FinishArgs f;
      f.mode = FIN_TCOL; f.partial = c->partial; f.nblk = nblk(ORTH_DOT); f.stride = orth_stride();
      f.T = c->T; f.ldT = SYEV_MAXB; f.cnt = j;
      S.check(fin(f), "fin refresh T");
    }
    return S.ok() ? TRPLK_OK : set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
  }

  // Block TRPL+K, one cycle's inner loop (readings B1-B4 of the block form):
  // the first block holds the preconditioned residuals of the targets t ..
  // t + nt - 1; each block is projected against [Q | U] by classical
  // Gram-Schmidt applied twice with block passes (one read of the basis for
  // every column), then its columns in order against the block's columns
  // already appended (the same, over those few columns), tested for
  // breakdown (R7) and appended; the appended columns are multiplied by A
  // together (one pass over A's diagonals) and turned into the next block,
  // M (A g - rho_j B g) with the shift of the target the column descends
  // from.  Host decisions per column (O(1) scalars read back); returns the
  // products with A it made.
  int block_inner(int t, int nt, int room, const double* shifts_host, long long* mv,
                  long long* precs) {
    Status S;
    const int bs = c->o.block;
    const double tol2 = std::pow(c->o.breakdown_tol > 0 ? c->o.breakdown_tol : BREAKDOWN_TOL, 2);
    const int next = c->prec == TRPLK_PREC_JACOBI ? NEXT_JACOBI
                     : c->prec == TRPLK_PREC_NONE ? NEXT_IDENT : NEXT_STORE_V;
    const bool fac = c->prec >= TRPLK_PREC_FSAI;
    HIPCHK(c, hipMemcpyAsync(c->bshift, shifts_host, sizeof(double) * nt, hipMemcpyHostToDevice, s));
    // first block: the targets' residuals through M
    std::vector<int> tgt(nt);
    for (int j = 0; j < nt; ++j) {
      tgt[j] = j;
      double* wj = c->Wblk + static_cast<int64_t>(j) * ld;
      S.check(restart_residual(n, AUcol(t + j), BUcol(t + j), c->bshift, j, next, c->dinv, wj,
                               fac ? c->vtmp : nullptr, nullptr, s), "block residual");
      if (fac) {
        S.check(apply_factor(), "block factor");
        S.check(copy_cols(n, c->w, ld, wj, ld, 1, s), "block copy");
      }
    }
    if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
    *precs += nt;
    int r = nt;
    std::vector<double> H1h(ORTH_MAXCOL * BLOCK_MAX), sm(4 * BLOCK_MAX);
    while (nbh < room && r > 0) {
      const int take = std::min(r, room - nbh);
      const int nq = c->u0 + nbh;   // columns of [Q | U]
      {
        // block CGS2 against [Q | U]: H1 = [BQ BU]^T W, W -= [Q U] H1, twice
        ProfScope ps(c, PC_ORTH, 4 * (8LL * n * nq) + 6 * 8LL * n * take);
        S.check(block_dot(n, nq, BWq(), ld, c->Wblk, ld, take, c->bpart, c->bh, ORTH_MAXCOL, s), "bdot1");
        S.check(hipMemcpyAsync(H1h.data(), c->bh, sizeof(double) * ORTH_MAXCOL * take,
                               hipMemcpyDeviceToHost, s), "h1 d2h");
        S.check(block_update(n, nq, Wq(), ld, c->bh, ORTH_MAXCOL, take, -1.0, c->Wblk, ld, s), "bupd1");
        S.check(block_dot(n, nq, BWq(), ld, c->Wblk, ld, take, c->bpart, c->bh, ORTH_MAXCOL, s), "bdot2");
        S.check(block_update(n, nq, Wq(), ld, c->bh, ORTH_MAXCOL, take, -1.0, c->Wblk, ld, s), "bupd2");
      }
      S.check(hipStreamSynchronize(s), "sync h1");
      if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
      const int nb0 = nbh;
      std::vector<int> nxt, kept;
      for (int j = 0; j < take; ++j) {
        double h1n2 = 0.0;
        for (int i = 0; i < nq; ++i) h1n2 += H1h[i + j * ORTH_MAXCOL] * H1h[i + j * ORTH_MAXCOL];
        double* wj = c->Wblk + static_cast<int64_t>(j) * ld;
        const int ja = nbh - nb0;   // block columns appended so far
        if (ja > 0) {
          // against the block's appended columns, twice (first-pass coefficients count in h1)
          S.check(block_dot(n, ja, BUcol(nb0), ld, wj, ld, 1, c->bpart, c->bsmall, BLOCK_MAX, s), "bdot3");
          S.check(block_update(n, ja, Ucol(nb0), ld, c->bsmall, BLOCK_MAX, 1, -1.0, wj, ld, s), "bupd3");
          S.check(hipMemcpyAsync(sm.data(), c->bsmall, sizeof(double) * ja, hipMemcpyDeviceToHost, s),
                  "h d2h");
          S.check(block_dot(n, ja, BUcol(nb0), ld, wj, ld, 1, c->bpart, c->bsmall + BLOCK_MAX,
                            BLOCK_MAX, s), "bdot4");
          S.check(block_update(n, ja, Ucol(nb0), ld, c->bsmall + BLOCK_MAX, BLOCK_MAX, 1, -1.0, wj, ld,
                               s), "bupd4");
        }
        // B-norm of the projected column
        const double* bw = wj;
        if (c->hasB) {
          SpmvArgs b;
          b.n = n; b.rowptr = c->B.rowptr; b.col = c->B.col; b.val = c->B.val; b.x = wj;
          b.mode = SPMV_STORE; b.y = c->tmpB;
          S.check(spmv(c->B, b, false, PC_SPMV, 0), "block B w");
          bw = c->tmpB;
        }
        S.check(block_dot(n, 1, wj, ld, bw, ld, 1, c->bpart, c->bsmall + 2 * BLOCK_MAX, 1, s), "bnorm");
        S.check(hipMemcpyAsync(sm.data() + 2 * BLOCK_MAX, c->bsmall + 2 * BLOCK_MAX, sizeof(double),
                               hipMemcpyDeviceToHost, s), "norm d2h");
        S.check(hipStreamSynchronize(s), "sync norm");
        if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
        for (int i = 0; i < ja; ++i) h1n2 += sm[i] * sm[i];
        const double beta2 = sm[2 * BLOCK_MAX];
        if (!std::isfinite(beta2)) return set_err(c, TRPLK_ENUMERIC, "non-finite block vector");
        if (!(beta2 > tol2 * (h1n2 + beta2))) continue;   // breakdown: the column is dropped
        const double ib = 1.0 / std::sqrt(beta2);
        S.check(scale_copy(n, ib, wj, Ucol(nbh), s), "append U");
        if (c->hasB) {
          S.check(scale_copy(n, ib, c->tmpB, BUcol(nbh), s), "append BU");
          ++bprod;
        }
        kept.push_back(j);
        ++*mv;
        ++nbh;
      }
      const int ra = nbh - nb0;
      // A g for the appended columns: one pass over A's diagonals for all of
      // them (SpMM), else one product per column
      if (ra > 0) {
        if (spmm_dia_ready(c->A.plan)) {
          ProfScope ps(c, PC_SPMV, spmv_matrix_bytes(c->A.plan, c->A.nnz, false) + 16LL * n * ra);
          S.check(spmm_dia(c->A.plan, n, Ucol(nb0), ld, ra, AUcol(nb0), ld, s), "block A G");
        } else {
          for (int q = 0; q < ra; ++q) {
            SpmvArgs a;
            a.n = n; a.rowptr = c->A.rowptr; a.col = c->A.col; a.val = c->A.val; a.x = Ucol(nb0 + q);
            a.mode = SPMV_STORE; a.y = AUcol(nb0 + q);
            S.check(spmv(c->A, a, false, PC_SPMV, 0), "block A g");
          }
        }
      }
      // the next block: column q from the q-th appended column with room
      // after it (index = number of columns kept so far; it only overwrites
      // columns of this block already consumed)
      for (int q = 0; q < ra && nb0 + q + 1 < room; ++q) {
        double* wq = c->Wblk + static_cast<int64_t>(q) * ld;
        S.check(restart_residual(n, AUcol(nb0 + q), BUcol(nb0 + q), c->bshift, tgt[kept[q]], next, c->dinv,
                                 wq, fac ? c->vtmp : nullptr, nullptr, s), "block next");
        if (fac) {
          S.check(apply_factor(), "block next factor");
          S.check(copy_cols(n, c->w, ld, wq, ld, 1, s), "block next copy");
        }
        nxt.push_back(tgt[kept[q]]);
        ++*precs;
      }
      // T columns of the appended block columns: T(0:nb0+j, nb0+j) = U^T A g_j
      if (ra > 0) {
        S.check(block_dot(n, nbh, Ucol(0), ld, AUcol(nb0), ld, ra, c->bpart, c->bh, ORTH_MAXCOL, s),
                "block T");
        S.check(block_tcols(c->bh, ORTH_MAXCOL, nb0, ra, c->T, SYEV_MAXB, s), "block T scatter");
      }
      if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
      tgt = nxt;
      r = static_cast<int>(nxt.size());
    }
    HIPCHK(c, set_state(c->st, SET_NB, 0.0, nbh, s));
    return TRPLK_OK;
  }
  long long bprod = 0;  // products with B made by the block inner loop

  int run(const double* x0, int32_t mem, trplk_stats* out);
  int run_pl1(const double* x0, int32_t mem, trplk_stats* out);
  void collect_profile();
};

int Solver::run(const double* x0, int32_t mem, trplk_stats* out) {
  const trplk_opts& o = c->o;
  const int p = o.p, m = o.m, k = o.k, l = o.l;
  const bool hard = c->pcap > 0;
  const double normA = (o.norm == TRPLK_NORM_FRO) ? c->normA_fro : c->normA_inf;
  const double thr = o.tol * normA;
  // float32 products carry errors of ~u32 ||A|| into T, large against a
  // clustered low spectrum, so the float32 phase ends early by default
  const double mixed_switch = (o.mixed_switch > 0 ? o.mixed_switch : 1e-3) * normA;
  double fp32_best = 0.0;  // float32 phase: best worst-target residual, its cycle and target
  int fp32_best_cycle = 0, fp32_target = -1;
  trplk_stats& stt = c->stats;
  stt = trplk_stats{};
  stt.a_ndiag = c->A.plan.ndiag;
  stt.b_ndiag = c->hasB ? c->B.plan.ndiag : 0;
  stt.g_ndiag = c->G.val ? c->G.plan.ndiag : 0;
  stt.normA = normA;
  c->prof.clear();
  c->evused = 0;
  c->u0 = 0;
  c->solved = false;
  c->fp32_phase = (o.precision == TRPLK_MIXED);
  c->hist.clear();
  const bool blk = o.block > 1;
  dc = o.orth != TRPLK_ORTH_CGS2 && !blk;
  stt.orth_delayed = dc ? 1 : 0;
  bprod = 0;
  int r;
  HIPCHK(c, hipEventRecord(c->ev0, s));
  HIPCHK(c, hipMemsetAsync(c->st, 0, sizeof(DevState), s));
  HIPCHK(c, hipMemsetAsync(c->T, 0, sizeof(double) * SYEV_MAXB * SYEV_MAXB, s));
  // ---- start block: B-orthonormalise X0 (Cholesky QR twice, or column by
  // column), A X0, T0 ----
  nbh = 0;
  r = (k >= CHOLQR_MIN_K && c->bpart) ? start_cholqr(x0, mem) : START_BY_COLUMNS;
  if (r != TRPLK_OK && r != START_BY_COLUMNS) return r;
  if (r == START_BY_COLUMNS) {
    HIPCHK(c, hipMemsetAsync(c->st, 0, sizeof(DevState), s));
    HIPCHK(c, hipMemsetAsync(c->T, 0, sizeof(double) * SYEV_MAXB * SYEV_MAXB, s));
    nbh = 0;
    for (int j = 0; j < k; ++j) {
      if ((r = load_w(x0 ? x0 + static_cast<int64_t>(j) * n : nullptr, mem, j))) return r;
      if ((r = add_vector(BREAKDOWN_TOL))) return r;
    }
  }
  if ((r = rayleigh_ritz(k, std::min(k, SYEV_MAXB)))) return r;
  if (c->rep_h->nb != k) return set_err(c, TRPLK_EINVAL, "start block is rank deficient");
  long long prev_app = c->rep_h->cnt_append;
  stt.matvecs = prev_app;
  std::vector<double> th(c->rep_h->theta, c->rep_h->theta + k);
  std::vector<double> res(c->rep_h->res, c->rep_h->res + k);
  std::vector<double> locked_theta;
  const int prec_saved = c->prec;
  const int window = o.fallback_window == 0 ? 50 : o.fallback_window;
  double best_res = 0.0;
  int best_cycle = 0, best_target = -1;
  int t = 0;         // target among the active Ritz pairs
  int kact = k;      // active Ritz vectors kept
  int nprev = 0;     // previous Ritz vectors held in Xprev
  int th_off = 0;    // index of the first active Ritz value in theta (device)
  bool done = false;
  int cycle = 0;
  for (cycle = 1; cycle <= o.max_cycles; ++cycle) {
    // ---- restart vector u1 = M (A x_t - rho B x_t) ----
    const double rho = th[t];
    HIPCHK(c, set_state(c->st, SET_RHO, rho, 0, s));
    HIPCHK(c, set_state(c->st, SET_NB, 0.0, kact, s));
    if (!keepT) HIPCHK(c, reset_T(c->T, SYEV_MAXB, SYEV_MAXB, kact, c->theta, th_off, s));
    keepT = false;
    nbh = kact;
    if (blk) {
      // ---- block TRPL+K: the inner blocks (B1-B4), then +K as below ----
      const int nt = std::max(1, std::min(o.block, kact - t));
      std::vector<double> sh(th.begin() + t, th.begin() + t + nt);
      long long mv = 0, pc = 0;
      if ((r = block_inner(t, nt, m - nprev, sh.data(), &mv, &pc))) return r;
      stt.matvecs += mv;
      stt.precs += pc;
    } else {
    {
      const bool fac = c->prec >= TRPLK_PREC_FSAI;
      const int next = c->prec == TRPLK_PREC_JACOBI ? NEXT_JACOBI
                       : c->prec == TRPLK_PREC_NONE ? NEXT_IDENT : NEXT_STORE_V;
      const bool f32v = fac && o.precision == TRPLK_MIXED;
      HIPCHK(c, restart_residual(n, AUcol(t), BUcol(t), c->theta, th_off + t, next, c->dinv, c->w,
                                 fac && !f32v ? c->vtmp : nullptr, f32v ? c->v32 : nullptr, s));
      if (fac) HIPCHK(c, apply_factor());
      stt.precs += 1;
    }
    // ---- inner preconditioned Krylov loop, eq. (3.1) ----
    const int m_in = m - kact - nprev;
    if ((r = stage_reset(o.breakdown_tol > 0 ? o.breakdown_tol : BREAKDOWN_TOL))) return r;
    if (dc) HIPCHK(c, set_identity(c->Lm, SYEV_MAXB, SYEV_MAXB, s));
    for (int j = 0; j < m_in; ++j) {
      const bool more = j < m_in - 1;
      if (dc) {
        // one Gram-Schmidt pass per vector before its product with A; the
        // second pass is the correction at the next step (the last vector's
        // is merged into the first +K vector's pass)
        if (j == 0 && (r = project_once())) return r;
        if ((r = append(more ? 1 : 0))) return r;
        if ((more || nprev == 0) && (r = dc_step(more))) return r;
      } else {
        if ((r = project(j == 0))) return r;
        if ((r = append(more ? 1 : 0))) return r;
        if ((r = tcol(more))) return r;
      }
      ++nbh;
      if (more) stt.precs += 1;
    }
    }  // scalar inner loop
    // ---- +K: previous Ritz vectors after the Krylov block ----
    if (dc && nprev > 0) {
      // each +K vector's single pass also corrects the pending column; the
      // last appended vector is corrected at the end
      for (int j = 0; j < nprev; ++j) {
        if ((r = stage_reset(PLUSK_DROP_TOL))) return r;
        if ((r = load_w(c->Xprev + j * ld, TRPLK_MEM_DEVICE, j))) return r;
        if ((r = dc_step(true, true))) return r;
        if ((r = append(0))) return r;
      }
      if ((r = dc_step(false, true))) return r;
      nbh += nprev;
    } else {
      for (int j = 0; j < nprev; ++j) {
        if ((r = load_w(c->Xprev + j * ld, TRPLK_MEM_DEVICE, j))) return r;
        if ((r = add_vector(PLUSK_DROP_TOL))) return r;
      }
    }
    HIPCHK(c, set_state(c->st, SET_SKIP, 0.0, 0, s));
    // previous vectors are taken from X before the Rayleigh-Ritz
    const int want = hard ? (p - c->u0) : p;
    const int lcnt = std::max(0, std::min(t + l, want) - t);
    HIPCHK(c, copy_cols(n, Ucol(t), ld, c->Xprev, ld, lcnt, s));
    // ---- Rayleigh-Ritz and thick restart ----
    const int kout = std::min(k, SYEV_MAXB);
    if ((r = rayleigh_ritz(kout, kout, dc))) return r;
    const Report& R = *c->rep_h;
    stt.matvecs += R.cnt_append - prev_app;
    prev_app = R.cnt_append;
    const int kk = std::min(kout, R.nb);
    th.assign(R.theta, R.theta + kk);
    c->hist.push_back(kk > 0 ? th[0] : NAN);
    res.assign(R.res, R.res + kk);
    nprev = lcnt;
    th_off = 0;
    if (!hard) {
      int tn = 0;
      while (tn < p && res[tn] <= thr) ++tn;
      if (tn > t) nprev = std::max(0, nprev - (tn - t));
      if (tn > t && nprev > 0) {
        // drop the first previous vector(s): shift the kept ones left
        const int drop = lcnt - nprev;
        HIPCHK(c, copy_cols(n, c->Xprev + drop * ld, ld, c->Xprev, ld, nprev, s));
      }
      t = tn;
      kact = kk;
      if (t >= p) {
        done = true;
        break;
      }
    } else {
      int nlock = 0;
      while (c->u0 + nlock < p && nlock < kk && res[nlock] <= thr) ++nlock;
      if (nlock) {
        for (int i = 0; i < nlock; ++i) locked_theta.push_back(th[i]);
        const int drop = std::min(nlock, nprev);
        nprev -= drop;
        if (drop && nprev > 0)
          HIPCHK(c, copy_cols(n, c->Xprev + drop * ld, ld, c->Xprev, ld, nprev, s));
        c->u0 += nlock;
        th.erase(th.begin(), th.begin() + nlock);
        res.erase(res.begin(), res.begin() + nlock);
        th_off = nlock;
      }
      t = 0;
      kact = kk - nlock;
      if (c->u0 >= p) {
        done = true;
        break;
      }
      if (kact <= 0) return set_err(c, TRPLK_EINVAL, "restart size exhausted by locking");
    }
    if (o.progress > 0 && cycle % o.progress == 0) {
      const int tt = hard ? 0 : std::min<int>(t, static_cast<int>(res.size()) - 1);
      std::fprintf(stderr, "trplk: cycle %d  converged %d/%d  target residual %.3e (threshold %.3e)  MV %lld\n",
                   cycle, hard ? c->u0 : t, p, res.empty() ? 0.0 : res[std::max(tt, 0)], thr,
                   static_cast<long long>(stt.matvecs));
      std::fflush(stderr);
    }
    // a factor preconditioner that stops making progress hands over to
    // Jacobi; the residuals (float64, true A and B) decide convergence
    if (window > 0 && c->prec >= TRPLK_PREC_FSAI) {
      const int target = hard ? c->u0 : t;
      const double rt = res.empty() ? 0.0 : res[hard ? 0 : std::min<int>(t, res.size() - 1)];
      if (target != best_target) {
        best_target = target;
        best_res = rt;
        best_cycle = cycle;
      } else if (rt < 0.5 * best_res) {
        best_res = rt;
        best_cycle = cycle;
      } else if (cycle - best_cycle >= window) {
        c->prec = TRPLK_PREC_JACOBI;
        stt.fallback_cycle = cycle;
      }
    }
    // mixed form: float64 SpMV once every target residual is small, or once
    // the float32 products stop the residual from falling (their error
    // floor can sit above the switch threshold)
    if (c->fp32_phase) {
      double worst = 0.0;
      for (int i = t; i < std::min<int>(static_cast<int>(res.size()), hard ? 1 : p); ++i)
        worst = std::max(worst, res[i]);
      const int target = hard ? c->u0 : t;
      if (target != fp32_target || worst < 0.5 * fp32_best) {
        fp32_target = target;
        fp32_best = worst;
        fp32_best_cycle = cycle;
      }
      const bool stalled = cycle - fp32_best_cycle >= MIXED_STALL_CYCLES;
      if (worst <= mixed_switch || stalled) {
        c->fp32_phase = false;
        stt.fp32_cycles = cycle;
        // theta on the device must hold the active values from index th_off
        if ((r = refresh_products(kact))) return r;
        stt.matvecs += kact;
        // T(0:kact,0:kact) now holds X^T A X; the next cycle keeps it
        keepT = true;
      }
    }
  }
  c->prec = prec_saved;
  if (cycle > o.max_cycles) cycle = o.max_cycles;
  stt.cycles = cycle;
  if (c->fp32_phase) stt.fp32_cycles = cycle;
  stt.bmatvecs = c->hasB ? c->rep_h->cnt_norm + bprod : 0;
  // ---- results ----
  if (hard) {
    // final Rayleigh-Ritz on the locked set: T_Q = Q^T A Q
    const int nq = c->u0;
    if (nq > 0) {
      Status S;
      for (int j = 0; j < nq; ++j) {
        OrthArgs a;
        a.n = n; a.ld = ld; a.ncol_fixed = j + 1; a.ncol_max = j + 1; a.Md0 = c->W;
        a.vec0 = c->AW + j * ld; a.nvec = 1; a.partial = c->partial;
        S.check(orth(ORTH_DOT, a), "TQ");
        FinishArgs f;
        f.mode = FIN_TCOL; f.partial = c->partial; f.nblk = nblk(ORTH_DOT); f.stride = orth_stride();
        f.T = c->T; f.ldT = SYEV_MAXB; f.cnt = j;
        S.check(fin(f), "fin TQ");
      }
      S.check(set_state(c->st, SET_NB, 0.0, nq, s), "nb");
      if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where);
      const int save = c->u0;
      c->u0 = 0;
      nbh = nq;
      r = rayleigh_ritz(nq, nq);
      c->u0 = save;
      if (r) return r;
    }
    c->theta_out.assign(c->rep_h->theta, c->rep_h->theta + std::min(nq, p));
    c->res_out.assign(c->rep_h->res, c->rep_h->res + std::min(nq, p));
    // not-yet-locked pairs fill the remainder
    for (int i = 0; static_cast<int>(c->theta_out.size()) < p && i < static_cast<int>(th.size()); ++i) {
      c->theta_out.push_back(th[i]);
      c->res_out.push_back(res[i]);
    }
    c->nout = std::min(p, nq + kact);
  } else {
    c->theta_out.assign(th.begin(), th.begin() + std::min<size_t>(p, th.size()));
    c->res_out.assign(res.begin(), res.begin() + std::min<size_t>(p, res.size()));
    c->nout = static_cast<int>(c->theta_out.size());
  }
  c->conv_out.assign(p, 0);
  int nconv = 0;
  for (int i = 0; i < static_cast<int>(c->res_out.size()); ++i) {
    c->conv_out[i] = c->res_out[i] <= thr;
    nconv += c->conv_out[i];
  }
  HIPCHK(c, hipEventRecord(c->ev1, s));
  HIPCHK(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  stt.solve_ms = ms;
  stt.nconv = nconv;
  stt.status = done ? TRPLK_OK : TRPLK_ENOCONV;
  collect_profile();
  c->solved = true;
  if (out) *out = stt;
  return stt.status;
}

void Solver::collect_profile() {
  trplk_stats& stt = c->stats;
  if (c->o.profile) {
    for (const Prof& pr : c->prof) {
      float e = 0.f;
      if (hipEventElapsedTime(&e, pr.a, pr.b) != hipSuccess) continue;
      switch (pr.cls) {
        case PC_SPMV: stt.spmv_ms += e; stt.spmv_launches++; stt.spmv_bytes += pr.bytes; break;
        case PC_DOT:
        case PC_UPDDOT:
        case PC_UPD:
        case PC_DCDOT:
        case PC_DCUPD: {
          stt.orth_ms += e; stt.orth_launches++; stt.orth_bytes += pr.bytes;
          const int q = pr.cls - PC_DOT;
          stt.pass_ms[q] += e; stt.pass_launches[q]++; stt.pass_bytes[q] += pr.bytes;
          break;
        }
        case PC_PREC: stt.prec_ms += e; stt.prec_launches++; stt.prec_bytes += pr.bytes; break;
        case PC_ROT: stt.rot_ms += e; stt.rot_launches++; stt.rot_bytes += pr.bytes; break;
        case PC_RR: stt.rr_ms += e; stt.rr_launches++; break;
      }
    }
  }
}

// PL+1 (Alg. 2, Sec. 4.2) for the smallest pair.  Per outer step: the
// preconditioned Krylov block G_k, B-orthonormal within itself (the first
// column x_k takes part in the T columns but not in the Gram-Schmidt
// coefficients), the previous search direction p_{k-1} appended with its
// stored products, the border of S = Q^T B Q from one dot pass, the lowest
// pair of the projected pencil (T, S) on the host, and one rotation of
// [Q, A Q, B Q] to [x_{k+1}, p_k].
int Solver::run_pl1(const double* x0, int32_t mem, trplk_stats* out) {
  const trplk_opts& o = c->o;
  const int m = o.m;
  const int mk = m - 2;
  const bool conj = o.method == TRPLK_METHOD_PL1;
  const double normA = (o.norm == TRPLK_NORM_FRO) ? c->normA_fro : c->normA_inf;
  const double thr = o.tol * normA;
  trplk_stats& stt = c->stats;
  stt = trplk_stats{};
  stt.a_ndiag = c->A.plan.ndiag;
  stt.b_ndiag = c->hasB ? c->B.plan.ndiag : 0;
  stt.g_ndiag = c->G.val ? c->G.plan.ndiag : 0;
  stt.normA = normA;
  c->prof.clear();
  c->evused = 0;
  c->u0 = 0;
  c->solved = false;
  c->fp32_phase = false;
  c->hist.clear();
  int r;
  HIPCHK(c, hipEventRecord(c->ev0, s));
  HIPCHK(c, hipMemsetAsync(c->st, 0, sizeof(DevState), s));
  HIPCHK(c, hipMemsetAsync(c->T, 0, sizeof(double) * SYEV_MAXB * SYEV_MAXB, s));
  // ---- x_0: B-normalised, A x_0, rho_0 = x_0^T A x_0, r_0 ----
  skip0 = 0;
  nbh = 0;
  if ((r = load_w(x0, mem, 0))) return r;
  if ((r = add_vector(BREAKDOWN_TOL))) return r;
  if ((r = rayleigh_ritz(1, 1))) return r;
  if (c->rep_h->nb != 1) return set_err(c, TRPLK_EINVAL, "start vector is zero");
  long long prev_app = c->rep_h->cnt_append;
  stt.matvecs = prev_app;
  double rho = c->rep_h->theta[0], res = c->rep_h->res[0], rho_prev = 0.0;
  bool have_p = false;
  bool done = res <= thr;
  int cycle = 0;
  skip0 = 1;
  while (!done && cycle < o.max_cycles) {
    ++cycle;
    HIPCHK(c, set_state(c->st, SET_RHO, rho, 0, s));
    HIPCHK(c, set_state(c->st, SET_NB, 0.0, 1, s));
    HIPCHK(c, reset_T(c->T, SYEV_MAXB, SYEV_MAXB, 1, c->theta, 0, s));
    nbh = 1;
    {  // u_1 = M r_k
      const bool fac = c->prec >= TRPLK_PREC_FSAI;
      const int next = c->prec == TRPLK_PREC_JACOBI ? NEXT_JACOBI
                       : c->prec == TRPLK_PREC_NONE ? NEXT_IDENT : NEXT_STORE_V;
      HIPCHK(c, restart_residual(n, AUcol(0), BUcol(0), c->theta, 0, next, c->dinv, c->w,
                                 fac ? c->vtmp : nullptr, nullptr, s));
      if (fac) HIPCHK(c, apply_factor());
      stt.precs += 1;
    }
    // ---- G_k: the preconditioned Krylov block (step 4) ----
    if ((r = stage_reset(BREAKDOWN_TOL))) return r;
    for (int j = 0; j < mk; ++j) {
      if ((r = project(j == 0))) return r;
      const bool more = j < mk - 1;
      if ((r = append(more ? 1 : 0))) return r;
      if ((r = tcol(more))) return r;
      ++nbh;
      if (more) stt.precs += 1;
    }
    HIPCHK(c, set_state(c->st, SET_SKIP, 0.0, 0, s));
    HIPCHK(c, hipMemcpyAsync(c->rep_h, c->st, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    int nq = c->rep_h->nb;  // 1 + columns of G_k kept
    // ---- Q_k = [x_k, G_k, p_{k-1}] (step 5) ----
    if (have_p) {
      Status S;
      S.check(copy_cols(n, c->Xprev, ld, Ucol(nq), ld, 1, s), "p");
      S.check(copy_cols(n, c->pl1_Ap, ld, AUcol(nq), ld, 1, s), "Ap");
      if (c->hasB) S.check(copy_cols(n, c->pl1_Bp, ld, BUcol(nq), ld, 1, s), "Bp");
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = nq + 1; a.ncol_max = nq + 1; a.Md0 = Ucol(0);
      a.vec0 = AUcol(nq); a.nvec = 1; a.partial = c->partial;
      S.check(orth(ORTH_DOT, a), "T p");
      FinishArgs f;
      f.mode = FIN_TCOL; f.partial = c->partial; f.nblk = nblk(ORTH_DOT); f.stride = orth_stride();
      f.T = c->T; f.ldT = SYEV_MAXB; f.cnt = nq;
      S.check(fin(f), "fin T p");
      if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where);
      ++nq;
    }
    {
      Status S;
      // border of S = Q^T B Q: rows of B x_k and B p_{k-1}
      OrthArgs a;
      a.n = n; a.ld = ld; a.ncol_fixed = nq; a.ncol_max = nq; a.Md0 = Ucol(0); a.Md1 = Ucol(0);
      a.vec0 = BUcol(0); a.vec1 = BUcol(nq - 1); a.nvec = 2; a.partial = c->partial;
      S.check(orth(ORTH_DOT, a), "S border");
      FinishArgs f;
      f.mode = FIN_SUM; f.partial = c->partial; f.nblk = nblk(ORTH_DOT); f.stride = orth_stride();
      f.out = c->pl1_s; f.cnt = ORTH_MAXCOL + nq;
      S.check(fin(f), "fin S border");
      // ---- lowest pair of Q^T A Q w = rho Q^T B Q w and the two rotation
      // columns (steps 5-7), on the device ----
      S.check(pl1_pencil(c->T, SYEV_MAXB, c->pl1_s, ORTH_MAXCOL, nq, have_p, conj, rho_prev, c->pl1_work,
                         c->pl1_q, c->Y, SYEV_MAXB, c->theta, c->st, s), "pencil");
      RotArgs ra;
      ra.n = n; ra.kout = 2; ra.state = c->st; ra.Y = c->Y; ra.ldY = SYEV_MAXB; ra.b_max = m;
      ra.U = Ucol(0); ra.AU = AUcol(0); ra.BU = c->hasB ? BUcol(0) : nullptr; ra.ld = ld;
      ra.theta = c->theta; ra.partial = c->partial;
      {
        const int64_t mats = c->hasB ? 3 : 2;
        ProfScope ps(c, PC_ROT, 8LL * n * (nq + 2) * mats);
        S.check(rotate(ra, c->rot_nblk, s), "rotate");
      }
      f = FinishArgs{};
      f.mode = FIN_RES; f.partial = c->partial; f.nblk = c->rot_nblk; f.stride = 128;
      f.out = c->resout; f.cnt = 1;
      S.check(fin(f), "fin res");
      // p_k and its products for the next step
      S.check(copy_cols(n, Ucol(1), ld, c->Xprev, ld, 1, s), "save p");
      S.check(copy_cols(n, AUcol(1), ld, c->pl1_Ap, ld, 1, s), "save Ap");
      if (c->hasB) S.check(copy_cols(n, BUcol(1), ld, c->pl1_Bp, ld, 1, s), "save Bp");
      hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, s, c->st, c->theta, c->resout, 1, 1,
                         c->rep_d);
      S.check(hipGetLastError(), "report");
      S.check(hipMemcpyAsync(c->rep_h, c->rep_d, sizeof(Report), hipMemcpyDeviceToHost, s), "d2h");
      S.check(hipStreamSynchronize(s), "sync");
      if (!S.ok()) return set_err(c, TRPLK_EDEVICE, S.where + ": " + hipGetErrorString(S.err));
    }
    switch (c->rep_h->pl1_err) {
      case 0: break;
      case 1: return set_err(c, TRPLK_ENOTSPD, "PL+1: projected B not positive definite");
      case 2: return set_err(c, TRPLK_ENUMERIC, "non-finite Ritz value");
      default: return set_err(c, TRPLK_ENUMERIC, "PL+1: zero direction");
    }
    const double lambda = c->rep_h->theta[0];
    if (c->rep_h->bad) return set_err(c, TRPLK_ENOTSPD, "B-norm squared not positive or not finite");
    stt.matvecs += c->rep_h->cnt_append - prev_app;
    prev_app = c->rep_h->cnt_append;
    have_p = true;
    rho_prev = rho;
    rho = lambda;
    c->hist.push_back(rho);
    res = c->rep_h->res[0];
    done = res <= thr;
  }
  skip0 = 0;
  stt.cycles = cycle;
  stt.bmatvecs = c->hasB ? c->rep_h->cnt_norm : 0;
  c->theta_out.assign(1, rho);
  c->res_out.assign(1, res);
  c->nout = 1;
  c->conv_out.assign(1, res <= thr ? 1 : 0);
  HIPCHK(c, hipEventRecord(c->ev1, s));
  HIPCHK(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  stt.solve_ms = ms;
  stt.nconv = done ? 1 : 0;
  stt.status = done ? TRPLK_OK : TRPLK_ENOCONV;
  collect_profile();
  c->solved = true;
  if (out) *out = stt;
  return stt.status;
}

}  // namespace

// ===================================================================== API
namespace {

int build_jacobi(trplk_ctx* c) {
  int* bad = nullptr;
  HIPCHK(c, dalloc(c, &c->dinv, c->n));
  HIPCHK(c, hipMalloc(&bad, sizeof(int)));
  HIPCHK(c, hipMemsetAsync(bad, 0, sizeof(int), c->s));
  HIPCHK(c, extract_diag_inv(c->n, c->A.rowptr, c->A.col, c->A.val, c->dinv, bad, c->s));
  int hb = 0;
  HIPCHK(c, hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  (void)hipFree(bad);
  if (hb) return set_err(c, TRPLK_ENOTSPD, "Jacobi: a diagonal entry of A is missing or not positive");
  return TRPLK_OK;
}

int compute_norms(trplk_ctx* c) {
  const int nb = rownorm_blocks(c->n);
  double* part = nullptr;
  HIPCHK(c, hipMalloc(&part, sizeof(double) * 2 * nb));
  HIPCHK(c, row_norms(c->n, c->A.rowptr, c->A.val, part, part + nb, nb, c->s));
  std::vector<double> h(2 * nb);
  HIPCHK(c, hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  (void)hipFree(part);
  double mx = 0.0, fr = 0.0;
  for (int i = 0; i < nb; ++i) {
    mx = std::max(mx, h[i]);
    fr += h[nb + i];
  }
  c->normA_inf = mx;
  c->normA_fro = std::sqrt(fr);
  return TRPLK_OK;
}

}  // namespace

namespace {

// G (device CSR owned by the context) -> G^T as CSR, float32 copies for the
// mixed form, SpMV plans.
int finish_factor(trplk_ctx* c) {
  DevCsr& G = c->G;
  DevCsr& Gt = c->Gt;
  Gt.n = G.n;
  Gt.nnz = G.nnz;
  Gt.owned = true;
  HIPCHK(c, csr_transpose(G.n, G.nnz, G.rowptr, G.col, G.val, &Gt.rowptr, &Gt.col, &Gt.val, c->s));
  c->dev_bytes += Gt.nnz * 12 + 4 * (Gt.n + 1);
  if (c->o.precision == TRPLK_MIXED) {
    HIPCHK(c, dalloc(c, &G.val32, std::max<int64_t>(G.nnz, 1)));
    HIPCHK(c, dalloc(c, &Gt.val32, std::max<int64_t>(Gt.nnz, 1)));
    HIPCHK(c, cast_f32(G.nnz, G.val, G.val32, c->s));
    HIPCHK(c, cast_f32(Gt.nnz, Gt.val, Gt.val32, c->s));
  }
  HIPCHK(c, spmv_plan(G.plan, G.n, G.rowptr, 0, c->s));
  HIPCHK(c, spmv_plan(Gt.plan, Gt.n, Gt.rowptr, 0, c->s));
  HIPCHK(c, spmv_plan_dia(G.plan, G.n, G.rowptr, G.col, G.val, G.val32, c->s));
  HIPCHK(c, spmv_plan_dia(Gt.plan, Gt.n, Gt.rowptr, Gt.col, Gt.val, Gt.val32, c->s));
  c->dev_bytes += dia_bytes(G.plan) + dia_bytes(Gt.plan);
  HIPCHK(c, hipStreamSynchronize(c->s));
  return TRPLK_OK;
}

}  // namespace

int trplk_internal_build_fsai(trplk_ctx* c) {
  free_csr(c->G);
  free_csr(c->Gt);
  int bad = 0;
  int64_t nnz = 0;
  HIPCHK(c, fsai_build(c->n, c->A.rowptr, c->A.col, c->A.val, c->o.fsai_cap, &c->G.rowptr,
                       &c->G.col, &c->G.val, &nnz, &bad, c->s));
  c->G.n = c->n;
  c->G.nnz = nnz;
  c->G.owned = true;
  c->dev_bytes += nnz * 12 + 4 * (c->n + 1);
  if (bad & 2)
    return set_err(c, TRPLK_EINVAL,
                   "FSAI: a row has more than 64 lower-triangular entries; set fsai_cap (<= 64)");
  if (bad) return set_err(c, TRPLK_ENOTSPD, "FSAI: missing diagonal or a local matrix is not SPD");
  return finish_factor(c);
}

int trplk_internal_set_factor(trplk_ctx* c, const trplk_csr* G, int32_t mem) {
  if (G->n != c->n) return set_err(c, TRPLK_EINVAL, "factor: dimension mismatch");
  if (mem == TRPLK_MEM_HOST) {
    std::string why;
    int r = validate_host_csr(G, c->n, why);
    if (r) return set_err(c, r, "factor: " + why);
    for (int i = 0; i < c->n; ++i) {
      const int e = G->rowptr[i + 1] - 1;
      if (e < G->rowptr[i] || G->col[e] != i)
        return set_err(c, TRPLK_EINVAL, "factor: not lower triangular with a diagonal entry");
      if (!(G->val[e] > 0.0)) return set_err(c, TRPLK_EINVAL, "factor: diagonal must be positive");
    }
  }
  free_csr(c->G);
  free_csr(c->Gt);
  DevCsr& D = c->G;
  D.n = c->n;
  D.nnz = G->nnz;
  D.owned = true;
  const hipMemcpyKind kd = mem == TRPLK_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  HIPCHK(c, dalloc(c, &D.rowptr, D.n + 1));
  HIPCHK(c, dalloc(c, &D.col, std::max<int64_t>(D.nnz, 1)));
  HIPCHK(c, dalloc(c, &D.val, std::max<int64_t>(D.nnz, 1)));
  HIPCHK(c, hipMemcpyAsync(D.rowptr, G->rowptr, sizeof(int) * (D.n + 1), kd, c->s));
  HIPCHK(c, hipMemcpyAsync(D.col, G->col, sizeof(int) * D.nnz, kd, c->s));
  HIPCHK(c, hipMemcpyAsync(D.val, G->val, sizeof(double) * D.nnz, kd, c->s));
  c->prec = TRPLK_PREC_FACTOR;
  return finish_factor(c);
}

// ------------------------------------------------------- learned factor --
namespace {

int learn_prepare(trplk_ctx* c) {
  auto& L = c->L;
  if (L.ready) return TRPLK_OK;
  const int n = c->n;
  hipStream_t s = c->s;
  int* cnt = nullptr;
  HIPCHK(c, hipMalloc(&cnt, sizeof(int) * (n + 1)));
  HIPCHK(c, hipMemsetAsync(cnt, 0, sizeof(int) * (n + 1), s));
  HIPCHK(c, tril_count(n, c->A.rowptr, c->A.col, cnt, s));
  HIPCHK(c, dalloc(c, &L.Lrow, n + 1));
  HIPCHK(c, exclusive_scan_i32(cnt, L.Lrow, n, s));
  (void)hipFree(cnt);
  int nnz = 0;
  HIPCHK(c, hipMemcpyAsync(&nnz, L.Lrow + n, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  L.nnz = nnz;
  HIPCHK(c, dalloc(c, &L.Lcol, nnz));
  HIPCHK(c, dalloc(c, &L.lr, nnz));
  HIPCHK(c, dalloc(c, &L.lval, nnz));
  HIPCHK(c, tril_fill(n, c->A.rowptr, c->A.col, c->A.val, L.Lrow, L.Lcol, L.lr, L.lval, s));
  // transpose of the pattern carrying the original positions
  double* iota = nullptr;
  HIPCHK(c, hipMalloc(&iota, sizeof(double) * std::max(nnz, 1)));
  HIPCHK(c, iota_values(nnz, iota, s));
  HIPCHK(c, csr_transpose(n, nnz, L.Lrow, L.Lcol, iota, &L.Trow, &L.Tcol, &L.permd, s));
  (void)hipFree(iota);
  c->dev_bytes += 16LL * nnz + 4LL * (n + 1);
  // features need 1 / a_ii
  int* bad = nullptr;
  HIPCHK(c, dalloc(c, &L.dinv, n));
  HIPCHK(c, hipMalloc(&bad, sizeof(int)));
  HIPCHK(c, hipMemsetAsync(bad, 0, sizeof(int), s));
  HIPCHK(c, extract_diag_inv(n, c->A.rowptr, c->A.col, c->A.val, L.dinv, bad, s));
  int hb = 0;
  HIPCHK(c, hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  (void)hipFree(bad);
  if (hb) return set_err(c, TRPLK_ENOTSPD, "learned factor: a diagonal entry is missing or <= 0");
  HIPCHK(c, dalloc(c, &L.F, static_cast<int64_t>(n) * MLP_NF));
  HIPCHK(c, dalloc(c, &L.Fz, static_cast<int64_t>(n) * MLP_NF));
  HIPCHK(c, dalloc(c, &L.scratch, mlp_scratch_doubles()));
  HIPCHK(c, mlp_features(n, c->A.rowptr, c->A.col, c->A.val, L.F, L.Fz, L.scratch, s));
  HIPCHK(c, dalloc(c, &L.gval, nnz));
  HIPCHK(c, dalloc(c, &L.gvalT, nnz));
  HIPCHK(c, dalloc(c, &L.P, MLP_NPARAM));
  HIPCHK(c, dalloc(c, &L.am, MLP_NPARAM));
  HIPCHK(c, dalloc(c, &L.av, MLP_NPARAM));
  HIPCHK(c, dalloc(c, &L.loss, 1));
  HIPCHK(c, dalloc(c, &L.grad, MLP_NPARAM));
  HIPCHK(c, dalloc(c, &L.part, static_cast<int64_t>(learn_blocks()) * MLP_NPARAM));
  HIPCHK(c, dalloc(c, &L.cbar, 1));
  HIPCHK(c, coupling_scale(L.nnz, L.lr, L.Lcol, L.lval, L.dinv, L.part, L.cbar, s));
  HIPCHK(c, hipStreamSynchronize(s));
  L.ready = true;
  return TRPLK_OK;
}

// Pair buffers sized for S pairs (grown when a later call asks for more): six
// n x S blocks, so a context trained on few pairs holds little memory.
int learn_alloc_pairs(trplk_ctx* c, int S) {
  auto& L = c->L;
  if (L.Er && L.pair_cap >= S) return TRPLK_OK;
  if (L.Er) {
    void* lp[] = {L.Er, L.Rr, L.Y, L.D, L.Uu, L.Z, L.coef, L.w, L.dout};
    for (void* q : lp) dfree(q);
    L.Er = L.Rr = L.Y = L.D = L.Uu = L.Z = L.coef = L.w = nullptr;
    L.dout = nullptr;
    L.pairs = false;
  }
  L.pair_cap = S;
  const int64_t nS = static_cast<int64_t>(c->n) * S;
  HIPCHK(c, dalloc(c, &L.Er, nS));
  HIPCHK(c, dalloc(c, &L.Rr, nS));
  HIPCHK(c, dalloc(c, &L.Y, nS));
  HIPCHK(c, dalloc(c, &L.D, nS));
  HIPCHK(c, dalloc(c, &L.Uu, nS));
  HIPCHK(c, dalloc(c, &L.Z, nS));
  HIPCHK(c, dalloc(c, &L.coef, 128));
  HIPCHK(c, dalloc(c, &L.w, LEARN_MAXS));
  HIPCHK(c, dalloc(c, &L.dout, L.nnz));
  return TRPLK_OK;
}

int learn_forward(trplk_ctx* c, const float* params_host) {
  auto& L = c->L;
  HIPCHK(c, hipMemcpyAsync(L.P, params_host, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, c->s));
  HIPCHK(c, mlp_forward(L.nnz, L.lr, L.Lcol, L.lval, L.Fz, L.dinv, L.cbar, L.P, L.gval, nullptr,
                        c->s));
  HIPCHK(c, gather_values(L.nnz, L.gval, L.permd, L.gvalT, c->s));
  return TRPLK_OK;
}

int learn_loss_grad_run(trplk_ctx* c) {
  auto& L = c->L;
  LearnArgs a;
  a.n = c->n; a.nnz = L.nnz; a.S = L.S; a.Lrow = L.Lrow; a.lc = L.Lcol; a.lr = L.lr;
  a.lval = L.lval; a.Trow = L.Trow; a.Tcol = L.Tcol; a.gval = L.gval; a.gvalT = L.gvalT;
  a.Fz = L.Fz; a.dinv = L.dinv; a.cbar = L.cbar; a.P = L.P; a.Rr = L.Rr; a.Er = L.Er; a.en = L.w; a.Y = L.Y;
  a.Q = L.D; a.Z = L.Z; a.Uz = L.Uu; a.coef = L.coef; a.dout = L.dout; a.part = L.part;
  a.loss = L.loss; a.grad = L.grad;
  HIPCHK(c, learn_loss_grad(a, c->s));
  return TRPLK_OK;
}

}  // namespace

extern "C" {

int trplk_learned_factor(trplk_ctx* c, const float* params) {
  if (!c || !params) return set_err(c, TRPLK_EINVAL, "null argument");
  int r;
  if ((r = learn_prepare(c))) return r;
  if ((r = learn_forward(c, params))) return r;
  auto& L = c->L;
  free_csr(c->G);
  free_csr(c->Gt);
  // the installed factor owns copies, so later training steps do not change it
  const int n = c->n;
  const int64_t nz = std::max<int64_t>(L.nnz, 1);
  DevCsr* both[2] = {&c->G, &c->Gt};
  const int* rp[2] = {L.Lrow, L.Trow};
  const int* cl[2] = {L.Lcol, L.Tcol};
  const double* vl[2] = {L.gval, L.gvalT};
  for (int q = 0; q < 2; ++q) {
    DevCsr& D = *both[q];
    D.n = n;
    D.nnz = L.nnz;
    D.owned = true;
    HIPCHK(c, dalloc(c, &D.rowptr, n + 1));
    HIPCHK(c, dalloc(c, &D.col, nz));
    HIPCHK(c, dalloc(c, &D.val, nz));
    HIPCHK(c, hipMemcpyAsync(D.rowptr, rp[q], sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, c->s));
    HIPCHK(c, hipMemcpyAsync(D.col, cl[q], sizeof(int) * L.nnz, hipMemcpyDeviceToDevice, c->s));
    HIPCHK(c, hipMemcpyAsync(D.val, vl[q], sizeof(double) * L.nnz, hipMemcpyDeviceToDevice, c->s));
  }
  if (c->o.precision == TRPLK_MIXED) {
    HIPCHK(c, dalloc(c, &c->G.val32, std::max<int64_t>(L.nnz, 1)));
    HIPCHK(c, dalloc(c, &c->Gt.val32, std::max<int64_t>(L.nnz, 1)));
    HIPCHK(c, cast_f32(L.nnz, c->G.val, c->G.val32, c->s));
    HIPCHK(c, cast_f32(L.nnz, c->Gt.val, c->Gt.val32, c->s));
  }
  HIPCHK(c, spmv_plan(c->G.plan, c->n, c->G.rowptr, 0, c->s));
  HIPCHK(c, spmv_plan(c->Gt.plan, c->n, c->Gt.rowptr, 0, c->s));
  HIPCHK(c, spmv_plan_dia(c->G.plan, c->n, c->G.rowptr, c->G.col, c->G.val, c->G.val32, c->s));
  HIPCHK(c, spmv_plan_dia(c->Gt.plan, c->n, c->Gt.rowptr, c->Gt.col, c->Gt.val, c->Gt.val32, c->s));
  c->dev_bytes += dia_bytes(c->G.plan) + dia_bytes(c->Gt.plan);
  HIPCHK(c, hipStreamSynchronize(c->s));
  c->prec = TRPLK_PREC_FACTOR;
  return TRPLK_OK;
}

int64_t trplk_factor_nnz(trplk_ctx* c) {
  if (!c) return -1;
  if (learn_prepare(c)) return -1;
  return c->L.nnz;
}

int trplk_factor_values(trplk_ctx* c, double* val, int32_t mem) {
  if (!c || !val) return set_err(c, TRPLK_EINVAL, "null argument");
  if (!c->L.ready) return set_err(c, TRPLK_EINVAL, "no learned factor");
  HIPCHK(c, hipMemcpyAsync(val, c->L.gval, sizeof(double) * c->L.nnz,
                           mem == TRPLK_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  return TRPLK_OK;
}

int trplk_factor_loss_grad(trplk_ctx* c, const float* params, int32_t S, const double* E,
                           const double* R, int32_t mem, double* loss, double* grad) {
  if (!c || !params || !E || !R || !loss || !grad) return set_err(c, TRPLK_EINVAL, "null argument");
  if (S < 1 || S > LEARN_MAXS) return set_err(c, TRPLK_EINVAL, "S must be in 1..64");
  int r;
  if ((r = learn_prepare(c)) || (r = learn_alloc_pairs(c, S))) return r;
  auto& L = c->L;
  const int n = c->n;
  const int64_t nS = static_cast<int64_t>(n) * S;
  const hipMemcpyKind k = mem == TRPLK_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  // column-major inputs staged through D / Uu, then transposed
  HIPCHK(c, hipMemcpyAsync(L.D, E, sizeof(double) * nS, k, c->s));
  HIPCHK(c, hipMemcpyAsync(L.Uu, R, sizeof(double) * nS, k, c->s));
  HIPCHK(c, to_rowmajor(n, S, L.D, n, L.Er, c->s));
  HIPCHK(c, to_rowmajor(n, S, L.Uu, n, L.Rr, c->s));
  L.S = S;
  L.pairs = false;  // these pairs are not the solver's
  HIPCHK(c, learn_colnorms(n, S, L.Er, L.part, L.w, c->s));
  if ((r = learn_forward(c, params))) return r;
  if ((r = learn_loss_grad_run(c))) return r;
  HIPCHK(c, hipMemcpyAsync(loss, L.loss, sizeof(double), hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipMemcpyAsync(grad, L.grad, sizeof(double) * MLP_NPARAM, hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  return TRPLK_OK;
}

int trplk_train_step(trplk_ctx* c, float* params, float* adam_m, float* adam_v, int32_t step,
                     double lr, int32_t S, double* loss, double* grad) {
  if (!c || !params || !adam_m || !adam_v) return set_err(c, TRPLK_EINVAL, "null argument");
  if (step < 1) return set_err(c, TRPLK_EINVAL, "step counts from 1");
  if (S < 1 || S > LEARN_MAXS || S > c->m) return set_err(c, TRPLK_EINVAL, "S must be in 1..min(64, m)");
  int r;
  if ((r = learn_prepare(c)) || (r = learn_alloc_pairs(c, S))) return r;
  auto& L = c->L;
  const int n = c->n;
  if (!L.pairs || L.S != S) {
    if (!c->solved) return set_err(c, TRPLK_EINVAL, "train_step harvests pairs from a completed solve");
    // pairs (u, A u): the first S stored basis columns and their products
    HIPCHK(c, to_rowmajor(n, S, c->W, c->ld, L.Er, c->s));
    HIPCHK(c, to_rowmajor(n, S, c->AW, c->ld, L.Rr, c->s));
    HIPCHK(c, learn_colnorms(n, S, L.Er, L.part, L.w, c->s));
    L.S = S;
    L.pairs = true;
  }
  if ((r = learn_forward(c, params))) return r;
  if ((r = learn_loss_grad_run(c))) return r;
  HIPCHK(c, hipMemcpyAsync(L.am, adam_m, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(L.av, adam_v, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, c->s));
  HIPCHK(c, adam_step(L.P, L.am, L.av, L.grad, step, static_cast<float>(lr), c->s));
  HIPCHK(c, hipMemcpyAsync(params, L.P, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipMemcpyAsync(adam_m, L.am, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipMemcpyAsync(adam_v, L.av, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, c->s));
  if (loss) HIPCHK(c, hipMemcpyAsync(loss, L.loss, sizeof(double), hipMemcpyDeviceToHost, c->s));
  if (grad)
    HIPCHK(c, hipMemcpyAsync(grad, L.grad, sizeof(double) * MLP_NPARAM, hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  return TRPLK_OK;
}

void trplk_default_opts(trplk_opts* o) {
  if (!o) return;
  *o = trplk_opts{};
  o->p = 1;
  o->m = 18;
  o->k = 8;
  o->l = 1;
  o->tol = 1e-8;
  o->norm = TRPLK_NORM_INF;
  o->max_cycles = 5000;
  o->precond = TRPLK_PREC_JACOBI;
  o->precision = TRPLK_FP64;
  o->locking = TRPLK_LOCK_AUTO;
  o->fsai_cap = 0;
  o->profile = 0;
  o->mixed_switch = 0.0;
  o->method = TRPLK_METHOD_TRPLK;
  o->orth = TRPLK_ORTH_AUTO;
  o->breakdown_tol = 0.0;
  o->seed = 12;
}

static int check_opts(const trplk_opts* o, int n, std::string& why) {
  if (o->method < TRPLK_METHOD_TRPLK || o->method > TRPLK_METHOD_PL1_PRACTICAL) {
    why = "bad method";
    return TRPLK_EINVAL;
  }
  if (o->method != TRPLK_METHOD_TRPLK) {
    if (o->p != 1) { why = "PL+1 computes one pair: p must be 1"; return TRPLK_EINVAL; }
    if (o->precision != TRPLK_FP64) { why = "PL+1 runs in float64"; return TRPLK_EINVAL; }
    if (!(3 <= o->m && o->m <= SYEV_MAXB && o->m <= n)) { why = "PL+1 needs 3 <= m <= min(n, 64)"; return TRPLK_EINVAL; }
    if (o->k < 1 || o->l < 0) { why = "k must be >= 1 and l >= 0"; return TRPLK_EINVAL; }
    if (!(o->tol > 0.0)) { why = "tol must be > 0"; return TRPLK_EINVAL; }
    if (o->max_cycles < 1) { why = "max_cycles must be >= 1"; return TRPLK_EINVAL; }
    if (o->precond < TRPLK_PREC_NONE || o->precond > TRPLK_PREC_FACTOR) { why = "bad precond"; return TRPLK_EINVAL; }
    if (o->fsai_cap < 0 || o->fsai_cap > 64) { why = "fsai_cap must be in 0..64"; return TRPLK_EINVAL; }
    if (o->block > 1) { why = "PL+1 has no block form"; return TRPLK_EINVAL; }
    return TRPLK_OK;
  }
  if (o->p < 1) { why = "p must be >= 1"; return TRPLK_EINVAL; }
  if (o->k < 1) { why = "k must be >= 1"; return TRPLK_EINVAL; }
  if (o->l < 0) { why = "l must be >= 0"; return TRPLK_EINVAL; }
  if (o->m > SYEV_MAXB) { why = "m must be <= 64"; return TRPLK_EINVAL; }
  if (!(o->k + o->l + 1 <= o->m && o->m <= n)) { why = "need k + l + 1 <= m <= n"; return TRPLK_EINVAL; }
  const bool hard = (o->locking == TRPLK_LOCK_HARD) || (o->locking == TRPLK_LOCK_AUTO && o->p > o->k);
  if (!hard && o->p > o->k) { why = "soft locking needs p <= k"; return TRPLK_EINVAL; }
  if (hard && (o->p + o->m > n || o->p > SYEV_MAXB || o->p + o->m > ORTH_MAXCOL)) {
    why = "hard locking needs p + m <= min(n, 128) and p <= 64";
    return TRPLK_EINVAL;
  }
  if (!(o->tol > 0.0)) { why = "tol must be > 0"; return TRPLK_EINVAL; }
  if (o->max_cycles < 1) { why = "max_cycles must be >= 1"; return TRPLK_EINVAL; }
  if (o->precond < TRPLK_PREC_NONE || o->precond > TRPLK_PREC_FACTOR) { why = "bad precond"; return TRPLK_EINVAL; }
  if (o->precision != TRPLK_FP64 && o->precision != TRPLK_MIXED) { why = "bad precision"; return TRPLK_EINVAL; }
  if (o->orth < TRPLK_ORTH_AUTO || o->orth > TRPLK_ORTH_DELAYED) { why = "bad orth"; return TRPLK_EINVAL; }
  if (!(o->breakdown_tol >= 0.0 && o->breakdown_tol < 1.0)) { why = "breakdown_tol must be in [0, 1)"; return TRPLK_EINVAL; }
  if (o->fsai_cap < 0 || o->fsai_cap > 64) { why = "fsai_cap must be in 0..64"; return TRPLK_EINVAL; }
  if (o->block < 0 || o->block > BLOCK_MAX) { why = "block must be in 0..16"; return TRPLK_EINVAL; }
  if (o->block > 1) {
    if (o->block > o->k) { why = "block must be <= k"; return TRPLK_EINVAL; }
    if (o->precision != TRPLK_FP64) { why = "block TRPL+K runs in float64"; return TRPLK_EINVAL; }
    if (o->orth == TRPLK_ORTH_DELAYED) { why = "block TRPL+K uses CGS2"; return TRPLK_EINVAL; }
  }
  return TRPLK_OK;
}

static int create_impl(trplk_ctx** out, const trplk_csr* A, const trplk_csr* B, const trplk_opts* o,
                       int32_t mem, void* stream, void* ws, int64_t ws_bytes) {
  if (!out) return set_err(nullptr, TRPLK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!A || !o) return set_err(nullptr, TRPLK_EINVAL, "A or opts is NULL");
  if (mem != TRPLK_MEM_HOST && mem != TRPLK_MEM_DEVICE) return set_err(nullptr, TRPLK_EINVAL, "bad mem");
  const int n = A->n;
  if (n < 1) return set_err(nullptr, TRPLK_EINVAL, "n must be >= 1");
  std::string why;
  int r = check_opts(o, n, why);
  if (r) return set_err(nullptr, r, why);
  if (mem == TRPLK_MEM_HOST) {
    if ((r = validate_host_csr(A, n, why))) return set_err(nullptr, r, "A: " + why);
    if (B && (r = validate_host_csr(B, n, why))) return set_err(nullptr, r, "B: " + why);
  } else {
    if (!A->rowptr || !A->col || !A->val) return set_err(nullptr, TRPLK_EINVAL, "A: null array");
    if (A->nnz < 0 || A->nnz >= (int64_t(1) << 31)) return set_err(nullptr, TRPLK_EINVAL, "A: nnz out of range");
    if (B && (!B->rowptr || !B->col || !B->val || B->n != n)) return set_err(nullptr, TRPLK_EINVAL, "B: bad");
  }
  trplk_ctx* c = new trplk_ctx();
  c->s = static_cast<hipStream_t>(stream);
  c->o = *o;
  c->n = n;
  c->hasB = B != nullptr;
  c->ws_base = ws;
  c->ws_size = ws_bytes;
  c->prec = o->precond;
  // setup time: host wall clock from here to the drained stream (uploads,
  // SpMV plans and diagonal copies, norms, preconditioner, workspace)
  const auto t_setup0 = std::chrono::steady_clock::now();
  auto fail = [&](int code) {
    std::string msg = c->err;
    trplk_destroy(c);
    return set_err(nullptr, code, msg);
  };
  const bool mixed = o->precision == TRPLK_MIXED;
  if ((r = upload_csr(c, c->A, A, mem, mixed))) return fail(r);
  if (B && (r = upload_csr(c, c->B, B, mem, false))) return fail(r);
  if ((r = compute_norms(c))) return fail(r);
  // the Jacobi diagonal is also the fallback of the factor preconditioners
  if ((r = build_jacobi(c))) return fail(r);
  if (c->prec == TRPLK_PREC_FSAI) {
    if ((r = trplk_internal_build_fsai(c))) return fail(r);
  } else if (c->prec == TRPLK_PREC_FACTOR) {
    // installed later by trplk_set_factor; Jacobi-equivalent until then
    c->err = "";
  }
  if ((r = ensure_workspace(c))) return fail(r);
  if (hipStreamSynchronize(c->s) != hipSuccess) return fail(set_err(c, TRPLK_EDEVICE, "sync"));
  c->stats.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                t_setup0).count();
  *out = c;
  return TRPLK_OK;
}

int trplk_create(trplk_ctx** out, const trplk_csr* A, const trplk_csr* B, const trplk_opts* o,
                 int32_t mem, void* stream) {
  return create_impl(out, A, B, o, mem, stream, nullptr, 0);
}

int64_t trplk_workspace_size(int32_t n, int32_t has_b, const trplk_opts* o) {
  if (!o || n < 1) return -1;
  std::string why;
  if (check_opts(o, n, why)) return -1;
  trplk_ctx tmp;
  tmp.n = n;
  tmp.hasB = has_b != 0;
  tmp.o = *o;
  return ws_bytes_needed(&tmp);
}

int trplk_create_ws(trplk_ctx** out, const trplk_csr* A, const trplk_csr* B, const trplk_opts* o,
                    int32_t mem, void* stream, void* workspace, int64_t workspace_bytes) {
  if (!workspace) return set_err(nullptr, TRPLK_EINVAL, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
    return set_err(nullptr, TRPLK_EINVAL, "workspace must be 256-byte aligned");
  if (A && o) {
    const int64_t need = trplk_workspace_size(A->n, B != nullptr, o);
    if (need < 0 || workspace_bytes < need)
      return set_err(nullptr, TRPLK_EINVAL, "workspace smaller than trplk_workspace_size()");
  }
  return create_impl(out, A, B, o, mem, stream, workspace, workspace_bytes);
}

int trplk_set_factor(trplk_ctx* c, const trplk_csr* G, int32_t mem) {
  if (!c || !G) return set_err(c, TRPLK_EINVAL, "null argument");
  return trplk_internal_set_factor(c, G, mem);
}

int trplk_solve(trplk_ctx* c, const double* x0, int32_t mem, trplk_stats* st) {
  if (!c) return set_err(nullptr, TRPLK_EINVAL, "ctx is NULL");
  if (mem != TRPLK_MEM_HOST && mem != TRPLK_MEM_DEVICE) return set_err(c, TRPLK_EINVAL, "bad mem");
  if (c->prec >= TRPLK_PREC_FSAI && !c->G.val) return set_err(c, TRPLK_EINVAL, "no factor installed");
  if (x0 && mem == TRPLK_MEM_HOST) {
    const int64_t ncols = c->o.method == TRPLK_METHOD_TRPLK ? c->o.k : 1;
    for (int64_t i = 0; i < static_cast<int64_t>(c->n) * ncols; ++i)
      if (!std::isfinite(x0[i])) return set_err(c, TRPLK_ENUMERIC, "non-finite start block");
  }
  int r = ensure_workspace(c);
  if (r) return r;
  c->L.pairs = false;
  Solver S{c, c->n, c->ld, c->s};
  const double setup = c->stats.setup_ms;
  const int prec0 = c->prec;
  r = c->o.method == TRPLK_METHOD_TRPLK ? S.run(x0, mem, st) : S.run_pl1(x0, mem, st);
  c->prec = prec0;  // a fallback inside the solve does not outlive it
  c->stats.setup_ms = setup;
  if (st) st->setup_ms = setup;
  return r;
}

int trplk_get_eigpairs(trplk_ctx* c, double* evals, double* evecs, double* resid, int32_t* conv,
                       int32_t mem) {
  if (!c) return set_err(nullptr, TRPLK_EINVAL, "ctx is NULL");
  if (!c->solved) return set_err(c, TRPLK_EINVAL, "no solve has completed");
  if (mem != TRPLK_MEM_HOST && mem != TRPLK_MEM_DEVICE) return set_err(c, TRPLK_EINVAL, "bad mem");
  const int p = c->o.p;
  const int nout = c->nout;
  const int n = c->n;
  const int64_t ld = c->ld;
  const bool host = mem == TRPLK_MEM_HOST;
  // Host staging lives until the stream has drained: every exit below goes
  // through done(), which synchronises before these vectors are released.
  std::vector<double> ev(p, NAN), rr(p, NAN);
  std::vector<int32_t> cv(p, 0);
  for (int i = 0; i < std::min<int>(p, c->theta_out.size()); ++i) ev[i] = c->theta_out[i];
  for (int i = 0; i < std::min<int>(p, c->conv_out.size()); ++i) cv[i] = c->conv_out[i];
  auto done = [&](int code, const char* what, hipError_t e) {
    (void)hipStreamSynchronize(c->s);
    if (code == TRPLK_OK) return TRPLK_OK;
    return set_err(c, code, std::string(what) + ": " + hipGetErrorString(e));
  };
#define GETCHK(call)                                               \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return done(TRPLK_EDEVICE, #call, e_);   \
  } while (0)
  if (evecs)
    GETCHK(hipMemcpy2DAsync(evecs, sizeof(double) * n, c->W, sizeof(double) * ld,
                            sizeof(double) * n, nout, host ? hipMemcpyDeviceToHost
                                                           : hipMemcpyDeviceToDevice, c->s));
  if (resid && nout > 0) {
    // true residuals ||A x - theta B x|| / ||x|| with fresh float64 products;
    // the Ritz values go to the context's own device buffer (no allocation)
    GETCHK(hipMemcpyAsync(c->thout, ev.data(), sizeof(double) * nout, hipMemcpyHostToDevice, c->s));
    double h[2];
    for (int i = 0; i < nout; ++i) {
      const double* x = c->W + i * ld;
      if (c->hasB) {
        SpmvArgs b;
        b.n = n; b.rowptr = c->B.rowptr; b.col = c->B.col; b.val = c->B.val; b.x = x;
        b.mode = SPMV_STORE; b.y = c->tmpB;
        GETCHK(spmv_f64(c->B.plan, b, c->s));
      }
      SpmvArgs a;
      a.n = n; a.rowptr = c->A.rowptr; a.col = c->A.col; a.val = c->A.val; a.x = x; a.xd = x;
      a.mode = SPMV_RESID; a.y = c->ytmp; a.bx = c->hasB ? c->tmpB : nullptr;
      a.partial = c->partial; a.theta = c->thout; a.theta_idx = i;
      GETCHK(spmv_f64(c->A.plan, a, c->s));
      FinishArgs f;
      f.mode = FIN_SUM; f.partial = c->partial; f.nblk = spmv_partial_blocks(c->A.plan); f.stride = 1;
      f.out = c->resout; f.cnt = 1;
      GETCHK(finish(f, c->s));
      OrthArgs o;
      o.n = n; o.ld = ld; o.ncol_fixed = 1; o.ncol_max = 1; o.Md0 = x; o.vec0 = x; o.nvec = 1;
      o.partial = c->partial;
      GETCHK(orth_pass(ORTH_DOT, o, orth_blocks(n, ORTH_DOT), c->s));
      FinishArgs g;
      g.mode = FIN_SUM; g.partial = c->partial; g.nblk = orth_blocks(n, ORTH_DOT); g.stride = orth_stride();
      g.out = c->resout + 1; g.cnt = 1;
      GETCHK(finish(g, c->s));
      GETCHK(hipMemcpyAsync(h, c->resout, 2 * sizeof(double), hipMemcpyDeviceToHost, c->s));
      GETCHK(hipStreamSynchronize(c->s));
      rr[i] = std::sqrt(h[0]) / std::sqrt(h[1]);
    }
  }
  if (host) {
    // host outputs: plain copies, nothing left in flight that reads ev/rr/cv
    if (evals) std::memcpy(evals, ev.data(), sizeof(double) * p);
    if (conv) std::memcpy(conv, cv.data(), sizeof(int32_t) * p);
    if (resid) std::memcpy(resid, rr.data(), sizeof(double) * p);
  } else {
    if (evals) GETCHK(hipMemcpyAsync(evals, ev.data(), sizeof(double) * p, hipMemcpyHostToDevice, c->s));
    if (conv) GETCHK(hipMemcpyAsync(conv, cv.data(), sizeof(int32_t) * p, hipMemcpyHostToDevice, c->s));
    if (resid) GETCHK(hipMemcpyAsync(resid, rr.data(), sizeof(double) * p, hipMemcpyHostToDevice, c->s));
  }
#undef GETCHK
  hipError_t e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return set_err(c, TRPLK_EDEVICE, std::string("sync: ") + hipGetErrorString(e));
  return TRPLK_OK;
}

int32_t trplk_get_history(trplk_ctx* c, double* theta1, int32_t cap) {
  if (!c) return set_err(nullptr, TRPLK_EINVAL, "ctx is NULL");
  if (!c->solved) return set_err(c, TRPLK_EINVAL, "no solve has completed");
  if (cap < 0 || (cap > 0 && !theta1)) return set_err(c, TRPLK_EINVAL, "bad history buffer");
  const int32_t nc = static_cast<int32_t>(c->hist.size());
  for (int32_t i = 0; i < std::min(cap, nc); ++i) theta1[i] = c->hist[i];
  return nc;
}

int64_t trplk_get_factor(trplk_ctx* c, int32_t* rowptr, int32_t* col, double* val, int32_t mem) {
  if (!c) return set_err(nullptr, TRPLK_EINVAL, "ctx is NULL");
  if (!c->G.val) return set_err(c, TRPLK_EINVAL, "no factor installed");
  if (mem != TRPLK_MEM_HOST && mem != TRPLK_MEM_DEVICE) return set_err(c, TRPLK_EINVAL, "bad mem");
  const int64_t nnz = c->G.nnz;
  if (!rowptr && !col && !val) return nnz;
  const hipMemcpyKind kd = mem == TRPLK_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (rowptr) HIPCHK(c, hipMemcpyAsync(rowptr, c->G.rowptr, sizeof(int32_t) * (c->n + 1), kd, c->s));
  if (col) HIPCHK(c, hipMemcpyAsync(col, c->G.col, sizeof(int32_t) * nnz, kd, c->s));
  if (val) HIPCHK(c, hipMemcpyAsync(val, c->G.val, sizeof(double) * nnz, kd, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  return nnz;
}

int64_t trplk_device_bytes(const trplk_ctx* c) { return c ? c->dev_bytes : 0; }

const char* trplk_last_error(const trplk_ctx* c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

void trplk_destroy(trplk_ctx* c) {
  if (!c) return;
  if (c->s) (void)hipStreamSynchronize(c->s);
  free_csr(c->A);
  free_csr(c->B);
  free_csr(c->G);
  free_csr(c->Gt);
  if (!c->ws_base) {
    std::vector<WsPiece> pcs;
    ws_pieces(c, pcs);
    for (const WsPiece& q : pcs) dfree(*q.ptr);
  }
  void* ptrs[] = {c->dinv, c->pl1_s, c->pl1_work, c->pl1_q, c->cq_flag, c->T, c->theta, c->Y, c->hbuf, c->cbuf, c->Lm, c->YA,
                  c->partial, c->resout, c->thout, c->st, c->rep_d, c->bpart, c->bh, c->bsmall,
                  c->bshift};
  for (void* p : ptrs) dfree(p);
  auto& L = c->L;
  void* lp[] = {L.Lrow, L.Lcol, L.lr, L.lval, L.Trow, L.Tcol, L.permd, L.dinv, L.F, L.Fz,
                L.gval, L.gvalT, L.P, L.am, L.av, L.Er, L.Rr, L.Y, L.D, L.Uu, L.Z, L.coef, L.w,
                L.dout, L.part, L.loss, L.grad, L.scratch, L.cbar};
  for (void* p : lp) dfree(p);
  if (c->rep_h) (void)hipHostFree(c->rep_h);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"

// --------------------------------------------------- kernel-level entries
namespace {

struct Scratch {
  double* buf = nullptr;
  size_t bytes = 0;
};
Scratch g_scratch;

double* kernel_scratch(size_t bytes) {
  if (bytes > g_scratch.bytes) {
    if (g_scratch.buf) (void)hipFree(g_scratch.buf);
    g_scratch.buf = nullptr;
    if (hipMalloc(&g_scratch.buf, bytes) != hipSuccess) {
      g_scratch.bytes = 0;
      return nullptr;
    }
    g_scratch.bytes = bytes;
  }
  return g_scratch.buf;
}

int kernel_err(hipError_t e) {
  if (e == hipSuccess) return TRPLK_OK;
  g_create_err = hipGetErrorString(e);
  return TRPLK_EDEVICE;
}

// Reduction scratch of trplk_gemv_t_noalloc: one row of partial sums per
// workgroup of the dot pass (at most NOALLOC_BLOCKS workgroups of
// 3 * ORTH_MAXCOL doubles).  Each device holds its own copy for the life of
// the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device.
constexpr int NOALLOC_BLOCKS = 256;
constexpr int64_t NOALLOC_DOUBLES = int64_t(NOALLOC_BLOCKS) * 3 * ORTH_MAXCOL;
__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAXDEV = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAXDEV] = {};

// Address of this device's scratch (looked up once per device, with the
// device current); nullptr with *err set on failure.
double* noalloc_scratch(hipError_t* err) {
  int dev = -1;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= NOALLOC_MAXDEV) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess || !p) {
      if (*err == hipSuccess) *err = hipErrorInvalidSymbol;
      return nullptr;
    }
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  return g_noalloc_ptr[dev];
}

}  // namespace

extern "C" {

int trplk_spmv(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
               const double* x, double* y, int32_t lanes, void* stream) {
  if (n < 0 || (n > 0 && (!rowptr || !col || !val || !x || !y))) return TRPLK_EINVAL;
  if (lanes != 0 && (lanes < 1 || lanes > 64 || (lanes & (lanes - 1)))) return TRPLK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SpmvPlan plan;
  hipError_t e = spmv_plan(plan, n, rowptr, lanes, s);
  if (e == hipSuccess && lanes == 0) e = spmv_plan_dia(plan, n, rowptr, col, val, nullptr, s);
  if (e != hipSuccess) {
    spmv_plan_free(plan);
    return kernel_err(e);
  }
  SpmvArgs a;
  a.n = n; a.rowptr = rowptr; a.col = col; a.val = val; a.x = x; a.y = y; a.mode = SPMV_STORE;
  e = spmv_f64(plan, a, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  spmv_plan_free(plan);
  return kernel_err(e);
}

int trplk_spmm(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val, const double* X,
               int64_t ldx, int32_t ncols, double* Y, int64_t ldy, void* stream) {
  if (n < 0 || ncols < 1 || ncols > 16 || (n > 0 && (!rowptr || !col || !val || !X || !Y)) || ldx < n ||
      ldy < n)
    return TRPLK_EINVAL;
  if (n == 0) return TRPLK_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SpmvPlan plan;
  hipError_t e = spmv_plan(plan, n, rowptr, 0, s);
  if (e == hipSuccess) e = spmv_plan_dia(plan, n, rowptr, col, val, nullptr, s);
  if (e == hipSuccess) {
    if (spmm_dia_ready(plan)) {
      e = spmm_dia(plan, n, X, ldx, ncols, Y, ldy, s);
    } else {
      for (int j = 0; j < ncols && e == hipSuccess; ++j) {
        SpmvArgs a;
        a.n = n; a.rowptr = rowptr; a.col = col; a.val = val; a.x = X + static_cast<int64_t>(j) * ldx;
        a.y = Y + static_cast<int64_t>(j) * ldy; a.mode = SPMV_STORE;
        e = spmv_f64(plan, a, s);
      }
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  spmv_plan_free(plan);
  return kernel_err(e);
}

int trplk_spmv_f32(int32_t n, const int32_t* rowptr, const int32_t* col, const float* val,
                   const float* x, float* y, int32_t lanes, void* stream) {
  if (n < 0 || (n > 0 && (!rowptr || !col || !val || !x || !y))) return TRPLK_EINVAL;
  if (lanes != 0 && (lanes < 1 || lanes > 64 || (lanes & (lanes - 1)))) return TRPLK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SpmvPlan plan;
  hipError_t e = spmv_plan(plan, n, rowptr, lanes, s);
  if (e == hipSuccess && lanes == 0) e = spmv_plan_dia(plan, n, rowptr, col, nullptr, val, s);
  if (e != hipSuccess) {
    spmv_plan_free(plan);
    return kernel_err(e);
  }
  SpmvArgs a;
  a.n = n; a.rowptr = rowptr; a.col = col; a.val = val; a.x = x; a.y = y; a.mode = SPMV_STORE;
  e = spmv_f32(plan, a, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  spmv_plan_free(plan);
  return kernel_err(e);
}

// the Gram-Schmidt passes load row pairs with 16-byte loads
static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int trplk_gemv_t(int32_t n, int32_t c, const double* U, int64_t ldu, const double* v, double* h,
                 void* stream) {
  if (n < 1 || c < 1 || c > ORTH_MAXCOL || ldu < n || !U || !v || !h) return TRPLK_EINVAL;
  if (ldu % 2 != 0 || !aligned16(U) || !aligned16(v)) return TRPLK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nblk = orth_blocks(n, ORTH_DOT);
  double* part = kernel_scratch(sizeof(double) * nblk * orth_stride());
  if (!part) return TRPLK_ENOMEM;
  OrthArgs a;
  a.n = n; a.ld = ldu; a.ncol_fixed = c; a.ncol_max = c; a.Md0 = U; a.vec0 = v; a.nvec = 1;
  a.partial = part;
  hipError_t e = orth_pass(ORTH_DOT, a, nblk, s);
  FinishArgs f;
  f.mode = FIN_SUM; f.partial = part; f.nblk = nblk; f.stride = orth_stride(); f.out = h; f.cnt = c;
  if (e == hipSuccess) e = finish(f, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return kernel_err(e);
}

int trplk_gemv_t_noalloc(int32_t n, int32_t c, const double* U, int64_t ldu, const double* v,
                         double* h, void* stream) {
  if (n < 1 || c < 1 || c > ORTH_MAXCOL || ldu < n || !U || !v || !h) return TRPLK_EINVAL;
  if (ldu % 2 != 0 || !aligned16(U) || !aligned16(v)) return TRPLK_EINVAL;
  const int nblk = orth_blocks(n, ORTH_DOT);
  if (static_cast<int64_t>(nblk) * orth_stride() > NOALLOC_DOUBLES) {
    g_create_err = "trplk_gemv_t_noalloc: the dot pass needs more partial rows than the static "
                   "scratch holds";
    return TRPLK_EINVAL;
  }
  hipError_t e = hipSuccess;
  double* part = noalloc_scratch(&e);
  if (!part) return kernel_err(e);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every workgroup writes its whole row of partials before the finish reads
  // it, so nothing left by an earlier call is read
  OrthArgs a;
  a.n = n; a.ld = ldu; a.ncol_fixed = c; a.ncol_max = c; a.Md0 = U; a.vec0 = v; a.nvec = 1;
  a.partial = part;
  e = orth_pass(ORTH_DOT, a, nblk, s);
  FinishArgs f;
  f.mode = FIN_SUM; f.partial = part; f.nblk = nblk; f.stride = orth_stride(); f.out = h; f.cnt = c;
  if (e == hipSuccess) e = finish(f, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return kernel_err(e);
}

int trplk_block_dot(int32_t n, int32_t c, const double* U, int64_t ldu, const double* V,
                    int64_t ldv, int32_t r, double* H, int32_t ldh, void* stream) {
  if (n < 1 || c < 1 || c > 128 || r < 1 || r > 16 || ldu < n || ldv < n || ldh < c || !U || !V ||
      !H)
    return TRPLK_EINVAL;
  if (ldu % 2 != 0 || !aligned16(U)) return TRPLK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* part = kernel_scratch(sizeof(double) * block_partial_doubles());
  if (!part) return TRPLK_ENOMEM;
  hipError_t e = block_dot(n, c, U, ldu, V, ldv, r, part, H, ldh, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return kernel_err(e);
}

int trplk_block_update(int32_t n, int32_t c, const double* U, int64_t ldu, const double* H,
                       int32_t ldh, int32_t r, double alpha, double* V, int64_t ldv, void* stream) {
  if (n < 1 || c < 1 || c > 128 || r < 1 || r > 16 || ldu < n || ldv < n || ldh < c || !U || !V ||
      !H)
    return TRPLK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = block_update(n, c, U, ldu, H, ldh, r, alpha, V, ldv, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return kernel_err(e);
}

int trplk_cgs_update_dot(int32_t n, int32_t c, const double* U, int64_t ldu, const double* h,
                         double* w, double* h2, void* stream) {
  if (n < 1 || c < 1 || c > ORTH_MAXCOL || ldu < n || !U || !h || !w || !h2) return TRPLK_EINVAL;
  if (ldu % 2 != 0 || !aligned16(U) || !aligned16(w)) return TRPLK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nblk = orth_blocks(n, ORTH_UPD_DOT);
  double* part = kernel_scratch(sizeof(double) * nblk * orth_stride());
  if (!part) return TRPLK_ENOMEM;
  OrthArgs a;
  a.n = n; a.ld = ldu; a.ncol_fixed = c; a.ncol_max = c; a.Mu = U; a.Md1 = U; a.h = h; a.w = w;
  a.partial = part;
  hipError_t e = orth_pass(ORTH_UPD_DOT, a, nblk, s);
  FinishArgs f;
  f.mode = FIN_SUM; f.partial = part; f.nblk = nblk; f.stride = orth_stride(); f.out = h2; f.cnt = c;
  if (e == hipSuccess) e = finish(f, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return kernel_err(e);
}

int trplk_syev(int32_t b, const double* T, double* theta, double* Y, void* stream) {
  if (b < 1 || b > SYEV_MAXB || !T || !theta || !Y) return TRPLK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = syev(T, b, b, nullptr, 0, theta, Y, b, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return kernel_err(e);
}

int trplk_rotate(int32_t n, int32_t b, int32_t k, double* U, int64_t ldu, const double* Y,
                 int32_t ldy, void* stream) {
  if (n < 1 || b < 1 || b > SYEV_MAXB || k < 1 || k > b || ldu < n || ldy < b || !U || !Y)
    return TRPLK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RotArgs a;
  a.n = n; a.kout = k; a.b_fixed = b; a.Y = Y; a.ldY = ldy; a.U = U; a.ld = ldu;
  hipError_t e = rotate(a, rot_blocks(n), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return kernel_err(e);
}

}  // extern "C"
