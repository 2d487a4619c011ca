// Shared device helpers and the internal launch interface of the TRPL+K
// library.  Everything here is gfx950-only HIP C++ (64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace trplk {

constexpr int WAVE = 64;

// Device-resident scalars of one solver context.  Kernels read the basis
// size from here so that a breakdown detected on the device stops the
// remaining launches of a stage without a host round trip.
struct DevState {
  int nb;          // columns of the active basis U (after the locked set)
  int skip;        // nonzero: step kernels of the current stage return at once
  int bad;         // nonzero: a B-norm squared <= 0 or a non-finite value was seen
  int pending;     // delayed form: column nb holds a vector awaiting its correction
  int arrive;      // workgroups of the running pass that are done (last-workgroup finish); 0 between passes
  double beta2;    // B-norm squared of the vector being appended
  double inv_beta; // 1 / sqrt(beta2)
  double h1norm2;  // squared norm of the first Gram-Schmidt coefficients
  double rho;      // shift of the inner operator
  double tol2;     // breakdown tolerance squared of the current stage
  long long cnt_append;  // vectors appended to the basis (one A product each)
  long long cnt_norm;    // B-norm evaluations (one B product each when B != I)
  double inv_gamma;      // delayed correction: 1 / ||u' - U c|| of the column being corrected
  int pl1_err;           // PL+1 projected pencil: 0 ok, 1 not positive definite, 2 non-finite, 3 zero direction
};

// Launch-error helper: records the first failing call.
struct Status {
  hipError_t err = hipSuccess;
  std::string where;
  bool ok() const { return err == hipSuccess; }
  void check(hipError_t e, const char* w) {
    if (e != hipSuccess && err == hipSuccess) {
      err = e;
      where = w;
    }
  }
};

// ---------------------------------------------------------------- device --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

template <int L>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, L);
  return v;
}

template <int L>
__device__ __forceinline__ float group_sumf(float v) {
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, L);
  return v;
}

// ------------------------------------------------------------ launchers --
// SpMV epilogues
enum SpmvMode : int {
  SPMV_STORE = 0,   // y = scale * A x (scale = 1 or state->inv_beta when use_beta)
  SPMV_APPEND = 1,  // append a basis vector: see SpmvArgs
  SPMV_DOT = 2,     // y = A x and a per-block partial of sum_i y_i x_i
  SPMV_RESID = 3    // y = A x - theta[j] * bx, and partial of ||y||^2 (true residual)
};

enum NextDir : int { NEXT_NONE = 0, NEXT_IDENT = 1, NEXT_JACOBI = 2, NEXT_STORE_V = 3 };

struct SpmvArgs {
  int n = 0;
  const int* rowptr = nullptr;
  const int* col = nullptr;
  const void* val = nullptr;    // double or float
  const void* x = nullptr;      // double or float gather vector
  int mode = SPMV_STORE;
  bool use_beta = false;        // scale by state->inv_beta
  bool out_f64 = false;         // float32 kernels: write y as float64
  DevState* state = nullptr;    // skip flag, inv_beta, rho, nb
  void* y = nullptr;            // SPMV_STORE/DOT/RESID output (double or float)
  // SPMV_APPEND: column nb (from state) of U, AU, BU is written with
  // inv_beta * (x_i, (A x)_i, bx_i); the next inner direction is formed
  // from v = inv_beta * ((A x)_i - rho * bx_i).
  const double* xd = nullptr;   // float64 copy of x (own-row reads)
  const double* bx = nullptr;   // B x (own-row), nullptr when B = I
  double* U = nullptr;
  double* AU = nullptr;
  double* BU = nullptr;
  int64_t ld = 0;
  int col0 = 0;                 // column of U where the active basis starts
  int next = NEXT_NONE;
  const double* dinv = nullptr; // Jacobi
  double* wout = nullptr;       // next direction (float64)
  float* vout32 = nullptr;      // NEXT_STORE_V in float32 (factor preconditioner input)
  double* vout = nullptr;       // NEXT_STORE_V in float64
  // SPMV_DOT / SPMV_RESID partials (one double per block)
  double* partial = nullptr;
  const double* theta = nullptr;
  int theta_idx = 0;
};

struct SpmvPlan {
  int n = 0;
  int lanes = 8;
  int nlong = 0;            // rows with more than LONG_ROW entries
  int* long_rows = nullptr; // device list of those rows
  int nblk_short = 0;       // grid of the short-row kernel
  int maxlen = 0;           // longest row
  int maxtile = 0;          // most entries in a 64-row tile
  int kmax = 0;             // CSR-stream entries per lane (8), 0: row-split kernels
  int tile_rows = 64;       // CSR-stream rows per wavefront tile (64, 32, 16, 8)
  bool adaptive = false;    // CSR-Adaptive blocks (+ long rows) for irregular matrices
  int nblocks = 0;          // adaptive blocks
  int2* blocks = nullptr;   // device [first row, end row) per block
  // diagonal storage (set by spmv_plan_dia when every entry lies on one of
  // at most DIA_MAXD diagonals and the format moves fewer bytes than CSR):
  // value of diagonal d at row i in dia_val[d * n + i] (0 where the
  // diagonal leaves the matrix or the pattern has no entry); offsets
  // ascending.  When ndiag > 0 the launches use these values, not the CSR.
  int ndiag = 0;
  int* dia_off = nullptr;       // device, ndiag column offsets (col - row)
  double* dia_val = nullptr;    // device, ndiag * n (float64 products)
  float* dia_val32 = nullptr;   // device, ndiag * n (float32 products)
  // x staged in LDS per 256-row chunk: the offsets fall into ncl clusters
  // (windows of 256 + span rows); diagonal d reads window entry doff[d] + row
  // - chunk start.  ncl = 0: no staging (the windows would not fit).
  int ncl = 0;
  int cl_lo[8] = {};
  int cl_len[8] = {};
  int cl_base[8] = {};
  int doff[32] = {};
  int lds_elems = 0;
  int nblk_dia = 0;             // grid of the diagonal kernel
};
constexpr int DIA_MAXD = 32;
constexpr int ADAPT_MAXNNZ = 512;  // entries per adaptive block (LDS per wavefront)
constexpr int LONG_ROW = 256;

int pick_lanes(double mean_len);
// Builds the plan (row-length binning) for a device CSR; allocates the long
// row list on the device.
hipError_t spmv_plan(SpmvPlan& plan, int n, const int* rowptr_dev, int lanes, hipStream_t s);
// Adds diagonal storage to a plan when the pattern qualifies (see
// SpmvPlan): the column pattern is inspected on the host, the values are
// scattered on the device from val64 and/or val32 (either may be null; the
// matching precision is then unavailable, and a launch in it fails).
// Must be called again whenever the CSR values change.
hipError_t spmv_plan_dia(SpmvPlan& plan, int n, const int* rowptr_dev, const int* col_dev,
                         const double* val64, const float* val32, hipStream_t s);
// Bytes one product reads and writes for the matrix itself (values, and
// indices for CSR) in the format the plan launches.
int64_t spmv_matrix_bytes(const SpmvPlan& plan, int64_t nnz, bool f32);
void spmv_plan_free(SpmvPlan& plan);
// Number of blocks a SPMV_DOT / SPMV_RESID launch writes partials for.
int spmv_partial_blocks(const SpmvPlan& plan);
hipError_t spmv_f64(const SpmvPlan& plan, const SpmvArgs& a, hipStream_t s);
hipError_t spmv_f32(const SpmvPlan& plan, const SpmvArgs& a, hipStream_t s);
// Y(:, j) = A X(:, j), j < ncols <= 16, for a plan with float64 diagonal
// storage (spmm_dia_ready): the values are read once for all columns; each
// column is bitwise the product spmv_f64 forms with SPMV_STORE.
bool spmm_dia_ready(const SpmvPlan& plan);
hipError_t spmm_dia(const SpmvPlan& plan, int n, const double* X, int64_t ldx, int ncols, double* Y,
                    int64_t ldy, hipStream_t s);

// ---------------------------------------------------------- orth passes --
enum OrthMode : int {
  ORTH_DOT = 0,      // h_v = M_v^T vec_v for NV vectors (v0 with Md0, v1 with Md1)
  ORTH_UPD_DOT = 1,  // w <- w - Mu h ; h2 = Md1^T w
  ORTH_UPD = 2,      // wout <- w - Mu h ; optional ||wout||^2 partial; optional f32 copy
  ORTH_UPD2 = 3      // delayed step: u <- (u' - U c) inv_gamma in place, then
                     // wout <- w - U h - u h_last (+ ||wout||^2, f32 copy); see k_upd2
};

struct OrthArgs {
  int n = 0;
  const double* Mu = nullptr;   // update matrix (column-major, ld)
  const double* Md0 = nullptr;  // dot matrix for vec0
  const double* Md1 = nullptr;  // dot matrix for vec1
  int64_t ld = 0;
  int ncol_fixed = 0;           // columns = ncol_fixed + (state ? state->nb : 0) + ncol_extra
  int ncol_extra = 0;
  int ncol_max = 0;             // upper bound of the column count (sizes the register tiles)
  const DevState* state = nullptr;
  const double* vec0 = nullptr;
  const double* vec1 = nullptr;
  // when non-null, vec0 = vec0_base + (vec0_col0 + state->nb) * ld (the
  // column just appended, located on the device)
  const double* vec0_base = nullptr;
  int vec0_col0 = 0;
  const double* vec1_base = nullptr;  // the same for vec1
  const double* vec2 = nullptr;       // ORTH_DOT with nvec = 3 (all against Md0)
  const double* h = nullptr;    // update coefficients (device)
  double* w = nullptr;          // vector updated in place (ORTH_UPD_DOT) / input (ORTH_UPD)
  double* wout = nullptr;       // ORTH_UPD output
  float* wout32 = nullptr;      // ORTH_UPD optional float32 copy
  bool norm = false;            // ORTH_UPD: partial of ||wout||^2
  double* partial = nullptr;    // [nblk][stride]
  int nvec = 1;                 // ORTH_DOT: 1, 2 or 3
  const double* c = nullptr;    // ORTH_UPD2: correction coefficients of the pending column
  // ORTH_UPD / ORTH_UPD2 with norm: the last workgroup to finish sums the
  // partials and takes the acceptance decision of FIN_NORM (needs state);
  // norm_dc is FIN_NORM's dc flag
  int fuse_norm = 0;
  int norm_dc = 0;
};

constexpr int ORTH_MAXCOL = 128;
int orth_blocks(int n, int mode);   // grid of a pass (its partial count)
int orth_blocks_max(int n);
int orth_blocks_dot3(int n);        // grid of the three-vector dot pass (nvec = 3)
int orth_stride();  // partial stride per block (doubles)
hipError_t orth_pass(int mode, const OrthArgs& a, int nblk, hipStream_t s);

// ------------------------------------------------------- finish kernels --
enum FinishMode : int {
  FIN_TH = 0,    // T column from vec0 dots + h1 from vec1 dots, nb += 1
  FIN_H = 1,     // h1 from vec0 dots (single vector)
  FIN_T = 2,     // T column from vec0 dots, nb += 1
  FIN_H2 = 3,    // h2 (update coefficients of the second pass)
  FIN_NORM = 4,  // beta^2: breakdown test, inv_beta, skip flag
  FIN_SUM = 5,   // plain sums into out[0..cnt)
  FIN_TCOL = 6,  // T column j = cnt from vec0 dots over columns 0..j, no state
  FIN_RES = 7,   // residual report: out[i] = sqrt(r2_i / x2_i), i < cnt (rotation partials)
  FIN_DC = 8     // delayed step: correction c, 1/gamma, corrected T column, h of the new
                 // direction (when nvec = 3), column of L; nb += 1
};

struct FinishArgs {
  int mode = FIN_SUM;
  const double* partial = nullptr;
  int nblk = 0;
  int stride = 0;
  DevState* state = nullptr;
  int ncol_fixed = 0;   // locked columns in front of U
  int extra = 0;        // 1 when the dot pass included the just-appended column
  double* T = nullptr;  // projected matrix, column-major, ldT
  int ldT = 0;
  double* h = nullptr;  // coefficient output (device, ORTH_MAXCOL)
  double* out = nullptr;
  int cnt = 0;
  int nvec = 1;
  int skip_first = 0;   // FIN_TH / FIN_H / FIN_H2: zero the coefficient of the first active
                        // column (a basis orthogonalised among its own columns only)
  double* cbuf = nullptr;  // FIN_DC: correction coefficients out (ORTH_MAXCOL)
  double* L = nullptr;     // FIN_DC: AU_true = AU_stored L (upper triangular, ldT)
  int dc = 0;              // FIN_NORM: an accepted vector becomes pending (delayed form);
                           // FIN_DC: correct column nb only if it is pending
};
hipError_t finish(const FinishArgs& f, hipStream_t s);

// ---------------------------------------------------- small kernels -----
hipError_t set_state(DevState* st, int which, double dv, int iv, hipStream_t s);
enum SetWhich : int {
  SET_RHO = 0, SET_TOL2 = 1, SET_NB = 2, SET_SKIP = 3, SET_RESET_STAGE = 4, SET_RHO_FROM = 5
};
hipError_t set_rho_from(DevState* st, const double* theta, int idx, hipStream_t s);
// T <- 0 except T(i,i) = theta[off + i] for i < kact
hipError_t reset_T(double* T, int ldT, int m, int kact, const double* theta, int off, hipStream_t s);
// YA = L Y for b = state->nb columns of the upper triangular L (both ld)
hipError_t ly_product(const double* L, const double* Y, double* YA, int ld, const DevState* st,
                      hipStream_t s);
// L <- I (m x m, leading dimension ld)
hipError_t set_identity(double* L, int ld, int m, hipStream_t s);

// r = AX(:,t) - theta_t BX(:,t) followed by the Jacobi / identity scale, or
// stored for the factor preconditioner (v, float32 or float64).
hipError_t restart_residual(int n, const double* AXt, const double* BXt, const double* theta,
                            int t, int next, const double* dinv, double* wout, double* vout,
                            float* vout32, hipStream_t s);

hipError_t copy_cols(int n, const double* src, int64_t lds, double* dst, int64_t ldd, int ncols,
                     hipStream_t s);
hipError_t cast_f32(int64_t n, const double* x, float* y, hipStream_t s);
hipError_t cast_f64(int64_t n, const float* x, double* y, hipStream_t s);

// Setup kernels
hipError_t extract_diag_inv(int n, const int* rowptr, const int* col, const double* val,
                            double* dinv, int* bad, hipStream_t s);
hipError_t row_norms(int n, const int* rowptr, const double* val, double* partial_inf,
                     double* partial_fro, int nblk, hipStream_t s);
int rownorm_blocks(int n);

// ------------------------------------------------------------- FSAI --
// FSAI factor of A on its (capped) lower pattern; allocates the output CSR.
// bad_host = 1 when a diagonal entry is missing or a local matrix is not SPD.
hipError_t fsai_build(int n, const int* rowptr, const int* col, const double* val, int cap,
                      int** g_rowptr, int** g_col, double** g_val, int64_t* g_nnz, int* bad_host,
                      hipStream_t s);
// CSR transpose with sorted columns (deterministic radix sort); allocates.
hipError_t csr_transpose(int n, int64_t nnz, const int* rowptr, const int* col, const double* val,
                         int** t_rowptr, int** t_col, double** t_val, hipStream_t s);

// ------------------------------------------------------ learned factor --
constexpr int MLP_NF = 8;                  // row features
constexpr int MLP_NIN = 2 * MLP_NF + 1;    // inputs per lower-triangular nonzero
constexpr int MLP_NH = 64;                 // hidden width
constexpr int MLP_NPARAM = MLP_NH * MLP_NIN + MLP_NH + MLP_NH + 1;  // W1, b1, w2, b2
constexpr int LEARN_MAXS = 64;             // training pairs per instance

struct LearnArgs {
  int n = 0;
  int64_t nnz = 0;            // lower-triangular nonzeros (G's pattern)
  int S = 0;
  const int* Lrow = nullptr;  // G row pointers
  const int* lc = nullptr;    // G columns
  const int* lr = nullptr;    // G row of each nonzero
  const double* lval = nullptr;  // a_ij on the pattern
  const int* Trow = nullptr;  // G^T row pointers / columns
  const int* Tcol = nullptr;
  const double* gval = nullptr;
  const double* gvalT = nullptr;
  const float* Fz = nullptr;
  const double* dinv = nullptr;
  const double* cbar = nullptr;  // mean normalised coupling (device scalar)
  const float* P = nullptr;   // parameters (device)
  const double* Rr = nullptr; // pairs, row-major n x S
  const double* Er = nullptr;
  const double* en = nullptr; // ||e_s||^2
  double* Y = nullptr;        // G r
  double* Q = nullptr;        // G^T G r
  double* Z = nullptr;
  double* Uz = nullptr;       // G z
  double* coef = nullptr;     // 128
  float* dout = nullptr;
  double* part = nullptr;     // learn_blocks() * MLP_NPARAM
  double* loss = nullptr;
  double* grad = nullptr;     // MLP_NPARAM
};

hipError_t mlp_features(int n, const int* rowptr, const int* col, const double* val, double* F,
                        float* Fz, double* scratch, hipStream_t s);
int mlp_scratch_doubles();
hipError_t tril_count(int n, const int* rowptr, const int* col, int* cnt, hipStream_t s);
hipError_t tril_fill(int n, const int* rowptr, const int* col, const double* val, const int* lrow,
                     int* lcol, int* lr, double* lval, hipStream_t s);
hipError_t mlp_forward(int64_t nnz, const int* lr, const int* lc, const double* lval,
                       const float* Fz, const double* dinv, const double* cbar, const float* P,
                       double* gval, float* oval, hipStream_t s);
// cbar = mean |a_ij| / sqrt(a_ii a_jj) over the strictly lower entries;
// part holds 2 * 256 doubles
hipError_t coupling_scale(int64_t nnz, const int* lr, const int* lc, const double* lval,
                          const double* dinv, double* part, double* cbar, hipStream_t s);
int learn_blocks();
hipError_t learn_loss_grad(const LearnArgs& a, hipStream_t s);
hipError_t learn_colnorms(int n, int S, const double* Er, double* part, double* en, hipStream_t s);
hipError_t adam_step(float* P, float* m, float* v, const double* grad, int t, float lr,
                     hipStream_t s);
hipError_t to_rowmajor(int n, int S, const double* Xc, int64_t ldx, double* Xr, hipStream_t s);
hipError_t gather_values(int64_t nnz, const double* src, const double* permd, double* dst,
                         hipStream_t s);
hipError_t iota_values(int64_t nnz, double* x, hipStream_t s);
hipError_t exclusive_scan_i32(const int* in, int* out, int n, hipStream_t s);

// ----------------------------------------------------------- eig / rot --
constexpr int SYEV_MAXB = 64;
// Jacobi eigensolver of T (b x b, b from *nb_dev or b_fixed when nb_dev is
// null), column-major with leading dimension ldT.
hipError_t syev(const double* T, int ldT, int b_fixed, const int* nb_dev, int nb_offset,
                double* theta, double* Y, int ldY, hipStream_t s);

// PL+1's projected pencil (pencil.hip): the lowest pair of (Q^T A Q, Q^T B Q)
// for Q = [x_k, G_k, p_{k-1}] (q = nq columns, p_{k-1} last when use_p; S: B
// inner products of x_k at S[0..nq) and of p_{k-1} at S[sp..sp+nq)), turned
// into the two rotation columns for x_{k+1} and p_k (Y, ld ldY), theta[0] =
// the Ritz value, st->nb = the columns used; failures in st->pl1_err.
// work: pl1_work_doubles() doubles, qdev: 2 ints (device).
int64_t pl1_work_doubles();
// Start block by Cholesky QR (pencil.hip): Rinv = R^-1 for G = R^T R (G
// k x k, symmetrised; flag = 1 when G is too close to singular), T <- (T +
// T^T)/2, and the state after k start vectors (nb, product counts).
hipError_t chol_inv(const double* G, int ldg, int k, double* Rinv, int ldr, int* flag, hipStream_t s);
hipError_t symmetrise(double* T, int ldT, int k, hipStream_t s);
hipError_t start_state(DevState* st, int k, bool with_b, hipStream_t s);
hipError_t pl1_pencil(const double* T, int ldT, const double* S, int sp, int nq, bool use_p, bool conj,
                      double rho_prev, double* work, int* qdev, double* Y, int ldY, double* theta,
                      DevState* st, hipStream_t s);

struct RotArgs {
  int n = 0;
  int kout = 0;                // requested output columns (min with b)
  int b_fixed = 0;             // basis columns when state is null
  int b_max = 0;               // upper bound of the basis columns (sizes the K loop)
  const DevState* state = nullptr;
  const double* Y = nullptr;   // ldY
  const double* YA = nullptr;  // optional coefficients for AU (ldY); Y when null
  int ldY = 0;
  double* U = nullptr;         // rotated in place
  double* AU = nullptr;        // optional
  double* BU = nullptr;        // optional
  int64_t ld = 0;
  const double* theta = nullptr;  // residual partials when non-null
  double* partial = nullptr;      // [nblk][2 * 64]: ||AX_i - th_i BX_i||^2, ||X_i||^2
};
int rot_blocks(int n);
hipError_t rotate(const RotArgs& a, int nblk, hipStream_t s);

// ----------------------------------------------------- block passes --
// H (ncols x r, leading dimension ldh) = M^T V for M n x ncols (ncols <= 128,
// 16-byte aligned, even ld) and V n x r (r <= 16); partial: at least
// block_partial_doubles() doubles.  V += alpha M H.
int block_dot_blocks(int n);
int64_t block_partial_doubles();
hipError_t block_dot(int n, int ncols, const double* M, int64_t ld, const double* V, int64_t ldv,
                     int r, double* partial, double* H, int ldh, hipStream_t s);
hipError_t block_update(int n, int ncols, const double* M, int64_t ld, const double* H, int ldh,
                        int r, double alpha, double* V, int64_t ldv, hipStream_t s);
// y = alpha x (n entries)
hipError_t scale_copy(int n, double alpha, const double* x, double* y, hipStream_t s);
// T(i, nb0 + j) = T(nb0 + j, i) = H(i, j), i <= nb0 + j, j < r
hipError_t block_tcols(const double* H, int ldh, int nb0, int r, double* T, int ldT, hipStream_t s);

}  // namespace trplk
