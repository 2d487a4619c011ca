/*
 * trplk.h -- C ABI of an MI355X (gfx950) implementation of TRPL+K, the
 * thick-restart preconditioned Lanczos method with locally optimal (+K)
 * restarting of Wu, Xue and Stathopoulos (arXiv 1711.10128).
 *
 * The library computes the p algebraically smallest eigenpairs of the pencil
 * A v = lambda B v with A symmetric and B symmetric positive definite
 * (paper, Sec. 1, eq. (1.1)); B = NULL means the standard problem B = I.
 * Eigenvectors are B-orthonormal.  Every step of the iteration runs in HIP
 * kernels on one GPU; the host only sequences launches and reads O(m)
 * scalars once per restart cycle.
 *
 * Conventions for every entry point:
 *  - return value: 0 = TRPLK_OK, > 0 = completed with a warning, < 0 = error;
 *    no C++ exception crosses the ABI.  After an error on a context,
 *    trplk_last_error() describes it.
 *  - matrices are square CSR, 0-based, int32 row pointers and column
 *    indices, columns sorted ascending within a row, no duplicates,
 *    float64 values, nnz < 2^31.  A must be symmetric (not checked).
 *  - dense blocks are column-major (Fortran order) with leading dimension n.
 *  - `mem` tells whether a pointer argument is host memory (TRPLK_MEM_HOST)
 *    or device memory of the current HIP device (TRPLK_MEM_DEVICE).
 *  - the caller owns every buffer it passes; the library owns the context
 *    and everything the context allocates.
 *  - one context is used by one host thread at a time; calls on one context
 *    are ordered on the context's stream.
 */
#ifndef TRPLK_H
#define TRPLK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TRPLK_OK 0
#define TRPLK_ENOCONV 1    /* max_cycles reached: partial results, per-pair flags */
#define TRPLK_EINVAL (-1)  /* bad sizes, options or CSR structure */
#define TRPLK_ENOMEM (-2)  /* device allocation failed */
#define TRPLK_ENOTSPD (-3) /* a B-norm squared <= 0, or a non-positive pivot in setup */
#define TRPLK_ENUMERIC (-4) /* NaN or Inf in the projected matrix or the Ritz values */
#define TRPLK_EDEVICE (-5) /* a HIP runtime call failed */

enum { TRPLK_MEM_HOST = 0, TRPLK_MEM_DEVICE = 1 };

/* preconditioner M, applied as z = M r (paper Sec. 2.2: M approximates
 * (A - rho I)^{-1}; the paper's incomplete factorisations are replaced by
 * these) */
enum {
  TRPLK_PREC_NONE = 0,   /* M = I */
  TRPLK_PREC_JACOBI = 1, /* M = diag(A)^{-1} */
  TRPLK_PREC_FSAI = 2,   /* M = G^T G, G the FSAI factor on tril(A), built on the GPU */
  TRPLK_PREC_FACTOR = 3  /* M = G^T G with G given by trplk_set_factor (learned) */
};
/* arithmetic of the operator products */
enum {
  TRPLK_FP64 = 0, /* everything in float64 */
  TRPLK_MIXED = 1 /* float32 preconditioner apply always; float32 SpMV while every
                     target residual is above the switch threshold, then float64
                     SpMV; orthogonalisation, projection, Rayleigh-Ritz and the
                     restart rotation always float64 */
};
enum { TRPLK_LOCK_AUTO = 0, TRPLK_LOCK_SOFT = 1, TRPLK_LOCK_HARD = 2 };
/* outer method */
enum {
  TRPLK_METHOD_TRPLK = 0,        /* TRPL+K, Alg. 1 */
  TRPLK_METHOD_PL1 = 1,          /* PL+1, Alg. 2 (Sec. 4.2): the smallest pair (p = 1); the
                                    Krylov block is B-orthonormal within itself, the search
                                    direction is made conjugate to the previous one with
                                    respect to A - rho(x_{k-1}) B (step 7) */
  TRPLK_METHOD_PL1_PRACTICAL = 2 /* PL+1 with p_k = g_k + p_{k-1} w(m+2), the combination the
                                    Ritz vector uses (end of Sec. 4.2) */
};
enum { TRPLK_NORM_INF = 0, TRPLK_NORM_FRO = 1 };
/* orthogonalisation of the inner (Krylov) vectors of TRPL+K.  Both make each
 * new basis vector orthogonal to the basis to working accuracy with classical
 * Gram-Schmidt applied twice; they differ in when the second pass runs. */
enum {
  TRPLK_ORTH_AUTO = 0,    /* DELAYED for TRPL+K (PL+1 keeps CGS2) */
  TRPLK_ORTH_CGS2 = 1,    /* both passes before the vector is appended: three passes over
                             the basis per inner step */
  TRPLK_ORTH_DELAYED = 2  /* the second pass of vector j is merged with the first pass of
                             vector j + 1 (one dot pass and one update pass per inner step);
                             the T column and the stored products A U are corrected from
                             small matrices, B U in the update pass (with hard locking the
                             terms U^T A Q c_Q, second order in the loss of orthogonality
                             to the converged Q, are left out) */
};

typedef struct trplk_csr {
  int32_t n;              /* rows = columns */
  int64_t nnz;            /* rowptr[n] */
  const int32_t* rowptr;  /* n + 1 */
  const int32_t* col;     /* nnz */
  const double* val;      /* nnz */
} trplk_csr;

/* Solver options.  The paper's symbols (Alg. 1): p wanted pairs, maximum
 * basis size q (here m), previous vectors l; the thick-restart size k >= p
 * is the paper's minimum restart size p-hat (Sec. 3).  Requirements:
 * 1 <= p, k + l + 1 <= m <= n, m <= 64; soft locking needs p <= k,
 * hard locking p + m <= n. */
typedef struct trplk_opts {
  int32_t p;          /* wanted eigenpairs */
  int32_t m;          /* maximum basis size */
  int32_t k;          /* thick-restart size (Ritz vectors kept) */
  int32_t l;          /* previous Ritz vectors appended (+K), 0 gives TRLan-like restarts */
  double tol;         /* stop when ||A x - theta B x||_2 / ||x||_2 <= tol * ||A||  (eq. (5.1)) */
  int32_t norm;       /* TRPLK_NORM_INF (default) or TRPLK_NORM_FRO (the paper's choice) */
  int32_t max_cycles; /* default 5000 (Sec. 5) */
  int32_t precond;    /* TRPLK_PREC_* */
  int32_t precision;  /* TRPLK_FP64 or TRPLK_MIXED */
  int32_t locking;    /* TRPLK_LOCK_AUTO: soft when p <= k, else hard */
  int32_t fsai_cap;   /* FSAI: keep at most this many entries per row of the factor (the
                         diagonal and the fsai_cap - 1 largest |a_ij|, j < i; ties to the
                         smaller column), 1..64.  0 = no cap: the whole lower pattern of
                         each row; trplk_create then fails with EINVAL when a row has more
                         than 64 lower-triangular entries (diagonal included) */
  int32_t profile;    /* 1 = time the SpMV and orthogonalisation kernels with HIP events */
  double mixed_switch; /* MIXED: switch SpMV to float64 once all target residuals are below
                          mixed_switch * ||A|| (or once they have not halved for 8 cycles:
                          the float32 error floor can sit above the threshold); 0 selects
                          the default 1e-3 */
  int32_t fallback_window; /* FSAI / FACTOR: when the target residual has not halved for this
                              many cycles, continue with Jacobi (M may change between cycles,
                              Sec. 3); 0 selects 50, negative disables */
  int32_t method;     /* TRPLK_METHOD_*.  PL+1 needs p = 1 and FP64; its projection space
                         [x_k, G_k, p_{k-1}] has at most m columns (Krylov block m - 2); the
                         start vector is the first column of x0; cycles = outer steps */
  int32_t orth;       /* TRPLK_ORTH_* (TRPL+K only; PL+1 always uses CGS2) */
  double breakdown_tol; /* TRPL+K inner loop: stop the Krylov block when a new vector's
                           (B-)norm squared is at most breakdown_tol^2 (|h|^2 + norm^2),
                           h its Gram-Schmidt coefficients; 0 selects 1e-14, must be < 1 */
  uint64_t seed;      /* start block drawn on the device when trplk_solve gets x0 = NULL: the
                         paper starts from a seeded uniform random block (Sec. 5; default 12).
                         Entry e of the column-major n x k block (e = column * n + row) is
                         b * 2^-52 - 1, b the top 53 bits of SplitMix64's e-th output:
                         mix(seed + (e + 1) * 0x9e3779b97f4a7c15) with mix(z) = z ^= z >> 30,
                         z *= 0xbf58476d1ce4e5b9, z ^= z >> 27, z *= 0x94d049bb133111eb,
                         z ^= z >> 31 (Steele, Lea and Flood, OOPSLA 2014), so any exact
                         implementation of that definition reproduces the block */
  int32_t progress;   /* > 0: TRPL+K writes one line to stderr every `progress` restart
                         cycles (cycle, converged pairs, target residual, products);
                         0 = silent */
  int32_t block;      /* block TRPL+K (the block form the paper leaves to future work,
                         Sec. 5.5): 0 or 1 = TRPL+K; s = 2..16 (s <= k, float64, CGS2)
                         targets the s lowest unconverged pairs per cycle, each with its own
                         shift, and grows the basis by blocks of s vectors
                         M (A g_j - theta_j B g_j), each block B-orthogonalised against the
                         basis with block passes (one read of the basis per block) and then
                         column by column within itself; +K, Rayleigh-Ritz, restart and
                         locking are TRPL+K's */
} trplk_opts;

typedef struct trplk_stats {
  int32_t cycles;      /* restart cycles run */
  int32_t nconv;       /* pairs meeting the tolerance at exit */
  int64_t matvecs;     /* products with A (the paper's MV count) */
  int64_t bmatvecs;    /* products with B */
  int64_t precs;       /* preconditioner applications */
  int32_t fp32_cycles; /* cycles that used the float32 SpMV (MIXED) */
  int32_t status;      /* TRPLK_OK or TRPLK_ENOCONV */
  int32_t fallback_cycle; /* cycle at which the preconditioner fell back to Jacobi, 0 = never */
  int32_t orth_delayed; /* 1 when the inner vectors used TRPLK_ORTH_DELAYED */
  double normA;        /* the ||A|| used in the stopping test */
  double solve_ms;     /* device time of trplk_solve (HIP events on the context stream) */
  double setup_ms;     /* wall time of trplk_create: CSR upload, SpMV plans (including the
                          host scan of the column pattern and the diagonal copies), norms,
                          preconditioner, workspace; the stream drained at both ends */
  /* kernel profile (opts.profile = 1): summed device time and launch count */
  double spmv_ms;      int64_t spmv_launches;     int64_t spmv_bytes;
  double orth_ms;      int64_t orth_launches;     int64_t orth_bytes;
  double prec_ms;      int64_t prec_launches;     int64_t prec_bytes;
  double rot_ms;       int64_t rot_launches;      int64_t rot_bytes;
  double rr_ms;        int64_t rr_launches;
  /* the orthogonalisation split by pass: [0] dots (T column + first
     coefficients, and the last correction of a DELAYED inner block),
     [1] fused update + dots, [2] update + norm, [3] DELAYED three-vector dots
     (correction, T column, coefficients of the new direction), [4] DELAYED
     correction + update */
  double pass_ms[5];   int64_t pass_launches[5];  int64_t pass_bytes[5];
  /* storage the products with A and B use: the number of diagonals when
     the matrix is held by diagonals (at most 32 distinct column offsets and
     at most 85% of the CSR bytes per product), 0 for CSR */
  int32_t a_ndiag;     int32_t b_ndiag;
  int32_t g_ndiag;     /* the same for the factor G of FSAI / FACTOR (0 also when none) */
  int32_t pad_;
} trplk_stats;

typedef struct trplk_ctx trplk_ctx;

/* Fill *o with defaults: p=1 m=18 k=8 l=1 tol=1e-8 norm=INF max_cycles=5000
 * precond=JACOBI precision=FP64 locking=AUTO fsai_cap=0 profile=0 method=TRPLK
 * orth=AUTO seed=12 (the settings of the paper's experiments, Sec. 5, with
 * its maxBasisSize 18 and minRestartSize 8). */
void trplk_default_opts(trplk_opts* o);

/* Create a solver context for the pencil (A, B) (paper eq. (1.1)).
 * A, B: CSR in host or device memory per `mem`; host arrays are copied to
 * the device, device arrays are referenced (they must outlive the context
 * and stay unchanged).  B == NULL: standard problem.  stream: a hipStream_t,
 * NULL = the null stream.  Builds the preconditioner (Jacobi diagonal or the
 * FSAI factor) and ||A|| on the device.  Errors: EINVAL, ENOMEM, ENOTSPD
 * (FSAI pivot <= 0), EDEVICE; *out is NULL on error. */
int trplk_create(trplk_ctx** out, const trplk_csr* A, const trplk_csr* B,
                 const trplk_opts* o, int32_t mem, void* stream);

/* Bytes of caller workspace trplk_create_ws needs for a pencil of order n
 * (has_b != 0: B != I) under options o: the basis W = [Q | U] (hard locking:
 * p + m columns, else m), A W, B W (has_b), the l previous Ritz vectors
 * (Sec. 3, +K) and the n-vectors of one inner step (eq. (3.1)), each column
 * padded to a multiple of 32 doubles and each piece to 256 bytes.  -1 when
 * the options are invalid for n. */
int64_t trplk_workspace_size(int32_t n, int32_t has_b, const trplk_opts* o);

/* trplk_create with the n-length solver workspace supplied by the caller (a
 * framework's allocator owns the memory): `workspace` is device memory of
 * the current device, 256-byte aligned, at least trplk_workspace_size(n,
 * B != NULL, o) bytes, owned by the caller and left untouched by
 * trplk_destroy; it must outlive the context and no other context may use
 * it at the same time.  The library still allocates the setup structures
 * (SpMV plans, diagonal copies, the preconditioner, host-copied CSR arrays)
 * and buffers of O(m^2) doubles and of one reduction partial per workgroup.
 * Errors: those of trplk_create, and EINVAL for a NULL, misaligned or too
 * small workspace. */
int trplk_create_ws(trplk_ctx** out, const trplk_csr* A, const trplk_csr* B,
                    const trplk_opts* o, int32_t mem, void* stream, void* workspace,
                    int64_t workspace_bytes);

/* Install the preconditioner M = G^T G (M approximates the inverse of the
 * shifted operator, paper Sec. 2.2; applied in the inner step as
 * M (A g - rho B g), eq. (3.1)) for G sparse lower triangular with a positive
 * diagonal (e.g. the learned factor); switches the context to
 * TRPLK_PREC_FACTOR.  G in host or device memory per `mem`; it is copied.
 * Errors: EINVAL when G is not n x n, or (host memory only) not lower
 * triangular, a diagonal entry missing or not positive.  A device-memory G
 * is taken as given: its structure is not checked. */
int trplk_set_factor(trplk_ctx* ctx, const trplk_csr* G, int32_t mem);

/* Run TRPL+K (paper Alg. 1 with eq. (3.1) and the +K placement of Sec. 3;
 * generalized form with B-inner products, Sec. 3 and Alg. 2).
 * x0: n x k start block, column-major, any full-rank block (it is
 * B-orthonormalised first); host or device per `mem`; NULL draws the block
 * on the device from opts.seed (see trplk_opts.seed).  PL+1 uses column 0.
 * st: optional, filled on return.  Returns OK when all p pairs converged,
 * ENOCONV after max_cycles (results are still available), or an error. */
int trplk_solve(trplk_ctx* ctx, const double* x0, int32_t mem, trplk_stats* st);

/* Copy the result of the last solve, the outputs theta_i, x_i of Alg. 1:
 * evals (p, ascending), evecs (n x p, column-major, B-orthonormal; may be
 * NULL), resid (p; the residual norms ||A x - theta B x||_2 / ||x||_2 of
 * eq. (5.1) recomputed with fresh float64 products; may be NULL), conv (p
 * flags: resid <= tol ||A||; may be NULL).  `mem` applies to every output.
 * A hard-locking solve stopped by max_cycles before the locked and active
 * vectors number p returns fewer pairs: the missing entries are NaN (evals,
 * resid), 0 (conv) and left unwritten (evecs).  Returns after the stream has
 * drained.  Errors: EINVAL before a successful solve or for a bad `mem`. */
int trplk_get_eigpairs(trplk_ctx* ctx, double* evals, double* evecs, double* resid,
                       int32_t* conv, int32_t mem);

/* ------------------------------------------------------------------------
 * Learned factor.  A two-layer MLP (float32) maps features of each
 * lower-triangular nonzero (i, j) of A to a scalar o_ij; the factor is
 * G(i,i) = exp(o_ii)/sqrt(a_ii), G(i,j) = -o_ij a_ij/(cbar a_jj sqrt(a_ii))
 * (j < i; cbar = mean |a_ij|/sqrt(a_ii a_jj) over the strictly lower
 * entries: up to cbar the scale of the first-order symmetric Gauss-Seidel
 * factor, 1/sqrt(a_jj) for a constant-coefficient stencil), so M =
 * G^T G is SPD by construction and a zero output layer reproduces Jacobi.
 * Inputs: [f_i (8), f_j (8), |a_ij|/sqrt(a_ii a_jj)], f = z-scored row
 * features (degree, a_ii, sum / mean / min / max / std of |a_ij|, j != i,
 * a_ii / sum).  Parameters: TRPLK_MLP_NPARAM floats packed as W1 (64 x 17,
 * row-major), b1 (64), w2 (64), b2 (1).  Not in the paper: it replaces the
 * paper's incomplete factorisations (Sec. 5.3-5.4) with a factor whose
 * values are learned; FSAI / Jacobi remain the fallbacks.
 * ------------------------------------------------------------------------ */
#define TRPLK_MLP_NPARAM 1217

/* Evaluate the MLP on the GPU for A's lower pattern and install M = G^T G
 * (switches the context to TRPLK_PREC_FACTOR).  params: host array. */
int trplk_learned_factor(trplk_ctx* ctx, const float* params);

/* Nonzeros of the learned factor's pattern (tril(A)); builds the pattern on
 * first use.  -1 on error. */
int64_t trplk_factor_nnz(trplk_ctx* ctx);

/* Values of the factor last evaluated by the MLP, in the CSR order of
 * tril(A) (trplk_factor_nnz entries). */
int trplk_factor_values(trplk_ctx* ctx, double* val, int32_t mem);

/* Loss L = (1/S) sum_s [1 - <M r_s, e_s>^2 / (||M r_s||^2 ||e_s||^2)], M = G^T G
 * (the squared sine of the angle between the preconditioned residual and the
 * correction; the inner Krylov space is invariant to the scale of M r), over
 * the pairs (E, R) (n x S, column-major, S <= 64, host or device per `mem`) and its
 * gradient with respect to the MLP parameters (grad: host, TRPLK_MLP_NPARAM
 * doubles), computed by the training kernels (float32 network, float64 pair
 * algebra, fixed-order reductions). */
int trplk_factor_loss_grad(trplk_ctx* ctx, const float* params, int32_t S, const double* E,
                           const double* R, int32_t mem, double* loss, double* grad);

/* One Adam step (Kingma and Ba, Algorithm 1: beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected moments; float32 state) on the pairs (u, A u)
 * the last trplk_solve on this context left in its basis (the first
 * S <= min(m, 64) stored columns and their products: the kept Ritz vectors
 * followed by the last cycle's inner Krylov vectors).  params, adam_m,
 * adam_v: host arrays of TRPLK_MLP_NPARAM floats, updated in place; step:
 * Adam step count (>= 1); loss: optional output (before the update); grad:
 * optional output of the TRPLK_MLP_NPARAM-double gradient the step used.
 * Call it on several contexts in turn to train on several problems. */
int trplk_train_step(trplk_ctx* ctx, float* params, float* adam_m, float* adam_v, int32_t step,
                     double lr, int32_t S, double* loss, double* grad);

/* Convergence history of the last solve: theta1[c] = the smallest Ritz
 * value of the active basis after the Rayleigh-Ritz of restart cycle c + 1
 * (Alg. 1; with hard locking the smallest not yet locked), or for PL+1 the
 * Rayleigh quotient rho(x_{c+1}) after outer step c + 1 (Alg. 2) -- the
 * rho(x_k) of the quasi-optimality ratio of Sec. 4.3.  Host
 * memory, at most cap values written.  Returns the number of cycles
 * recorded, or a negative status (EINVAL before a completed solve). */
int32_t trplk_get_history(trplk_ctx* ctx, double* theta1, int32_t cap);

/* The factor G of the installed preconditioner M = G^T G (Sec. 2.2: M
 * approximates the inverse of the shifted operator): the FSAI factor built
 * by trplk_create, the learned factor or the one given to trplk_set_factor,
 * as CSR (n + 1 row pointers, nnz columns sorted within a row, nnz values;
 * host or device memory per `mem`).  With rowptr, col and val all NULL it
 * only returns nnz.  Returns nnz, or a negative status (EINVAL when no
 * factor is installed). */
int64_t trplk_get_factor(trplk_ctx* ctx, int32_t* rowptr, int32_t* col, double* val,
                         int32_t mem);

/* Bytes of device memory the context holds (matrices, preconditioner and the
 * solver workspace sized for its options). */
int64_t trplk_device_bytes(const trplk_ctx* ctx);

/* Human-readable description of the last error on ctx (or of the last
 * failed trplk_create when ctx is NULL). */
const char* trplk_last_error(const trplk_ctx* ctx);

/* Release the context and every device buffer it allocated (not a caller
 * workspace); waits for the context stream first.  NULL is a no-op. */
void trplk_destroy(trplk_ctx* ctx);

/* ------------------------------------------------------------------------
 * Kernel-level entry points.  Each runs one building block of the iteration
 * on device buffers (device pointers, hipStream_t `stream`, NULL = null
 * stream), so it can be checked and timed in isolation.  They allocate a
 * small reduction scratch on first use (kept until process exit); calls from
 * several host threads at once are not supported.
 * ------------------------------------------------------------------------ */

/* y = A x, CSR SpMV (the paper's matrix-vector product "MV", eq. (3.1)),
 * float64.  lanes: lanes of a wavefront per row (1,2,4,8,16,32,64), 0 = pick
 * from the mean row length.  Rows longer than 256 entries go to a
 * workgroup-per-row kernel. */
int trplk_spmv(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
               const double* x, double* y, int32_t lanes, void* stream);

/* Y(:, j) = A X(:, j) for j < ncols <= 16 (column-major X and Y, leading
 * dimensions ldx, ldy >= n), float64: the products with A of the columns a
 * block of block TRPL+K has appended (the block form the paper leaves to
 * future work, Sec. 5.5).  When A's pattern fits diagonal storage its values
 * are read once for all columns; each column equals trplk_spmv's product
 * (lanes = 0) bit for bit.  Other patterns take one CSR product per column.
 * Device pointers; EINVAL for ncols outside 1..16 or short leading
 * dimensions. */
int trplk_spmm(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val, const double* X,
               int64_t ldx, int32_t ncols, double* Y, int64_t ldy, void* stream);

/* Same in float32 (values, vector and accumulation): the SpMV of the
 * mixed-precision form. */
int trplk_spmv_f32(int32_t n, const int32_t* rowptr, const int32_t* col, const float* val,
                   const float* x, float* y, int32_t lanes, void* stream);

/* h = U^T v for U n x c (column-major, leading dimension ldu), c <= 128:
 * the projection coefficients of the Gram-Schmidt step (Sec. 3).  Device
 * pointers; U and v must be 16-byte aligned and ldu even (the pass loads
 * row pairs), otherwise TRPLK_EINVAL. */
int trplk_gemv_t(int32_t n, int32_t c, const double* U, int64_t ldu, const double* v,
                 double* h, void* stream);

/* trplk_gemv_t for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same h = U^T v with the same kernels and summation order, but the
 * per-workgroup partial sums go to a static device array of the library
 * (256 workgroups x 384 doubles = 768 KiB per device, held until the
 * process ends; its address is looked up once per device) instead of
 * memory the library allocates.  No hipMalloc, hipFree or allocating
 * library call is made.  Same arguments, layout and alignment rules as
 * trplk_gemv_t; TRPLK_EINVAL when the pass would need more partial rows
 * than the array holds.  Every call on one device shares that array: calls
 * that overlap on one GPU (several streams or host threads) race. */
int trplk_gemv_t_noalloc(int32_t n, int32_t c, const double* U, int64_t ldu, const double* v,
                         double* h, void* stream);

/* w <- w - U h followed by h2 = U^T w (one read of U): the fused second
 * pass of classical Gram-Schmidt applied twice.  Same layout and alignment
 * rules as trplk_gemv_t (U and w 16-byte aligned, ldu even). */
int trplk_cgs_update_dot(int32_t n, int32_t c, const double* U, int64_t ldu, const double* h,
                         double* w, double* h2, void* stream);

/* Block Gram-Schmidt passes of block TRPL+K (the block form the paper leaves
 * to future work, Sec. 5.5): H = U^T V for U n x c (c <= 128, column-major,
 * leading dimension ldu, 16-byte aligned, ldu even) and V n x r (r <= 16,
 * leading dimension ldv); H is c x r with leading dimension ldh.  One read
 * of U serves all r vectors (FP64 matrix cores).  Device pointers. */
int trplk_block_dot(int32_t n, int32_t c, const double* U, int64_t ldu, const double* V,
                    int64_t ldv, int32_t r, double* H, int32_t ldh, void* stream);

/* V <- V + alpha U H (U n x c, H c x r, V n x r; the same layout rules
 * except alignment): the block update of Gram-Schmidt (alpha = -1). */
int trplk_block_update(int32_t n, int32_t c, const double* U, int64_t ldu, const double* H,
                       int32_t ldh, int32_t r, double alpha, double* V, int64_t ldv, void* stream);

/* Symmetric eigendecomposition of a b x b matrix T (column-major, b <= 64),
 * ascending eigenvalues theta (b) and orthonormal eigenvectors Y (b x b):
 * the Rayleigh-Ritz step on the projected matrix (Alg. 1).  Device pointers. */
int trplk_syev(int32_t b, const double* T, double* theta, double* Y, void* stream);

/* In-place basis rotation U(:, 0:k) <- U(:, 0:b) * Y(:, 0:k) for U n x b
 * (leading dimension ldu), Y b x b column-major (leading dimension ldy),
 * k <= b <= 64: the thick restart X = U Y (Alg. 1).  Uses FP64 MFMA. */
int trplk_rotate(int32_t n, int32_t b, int32_t k, double* U, int64_t ldu, const double* Y,
                 int32_t ldy, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TRPLK_H */
