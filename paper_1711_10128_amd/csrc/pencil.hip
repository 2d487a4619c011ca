// PL+1's projected pencil on the device (Alg. 2, steps 5-7).
//
// Q_k = [x_k, G_k, p_{k-1}] has q <= 64 columns.  The projected matrices
// are TA = Q^T A Q (the symmetrised T the inner loop assembles) and
// TB = Q^T B Q, which is the identity except for its first row and column
// (x_k is not orthogonalised against G_k) and, when p_{k-1} is present, its
// last ones; both borders come from one dot pass.  The lowest pair of
// TA w = lambda TB w is found by the Cholesky reduction TB = L L^T,
// C = L^-1 TA L^-T, the eigenpairs of C (k_syev, the Rayleigh-Ritz solver
// of TRPL+K) and w = L^-T y.  If TB is numerically singular with p_{k-1}
// included (p_{k-1} almost in span{x_k, G_k}), p_{k-1} is dropped and the
// leading (q - 1) x (q - 1) pencil is used.
//
// From w the next iterate and search direction follow: the coordinates of
// x_{k+1} are w; those of the direction are w with the x_k entry zeroed
// (the G_k part), plus, with p_{k-1} present, either w's own p entry (the
// practical direction of Sec. 4.2) or the coefficient that makes the
// direction conjugate to p_{k-1} with respect to A - rho_{k-1} B (step 7).
// Both columns are B-normalised in the projected inner product and written
// as the two columns of the rotation that forms x_{k+1} and p_k.
//
// Three single-workgroup kernels, no host round trip: k_pl1_reduce,
// k_syev, k_pl1_direction.  Failures are recorded in DevState::pl1_err (1:
// TB not positive definite, 2: non-finite Ritz value, 3: a zero direction)
// for the host to read with the step's report.  The file also holds the
// small factorisation of the start block's Cholesky QR (k_chol_inv).
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"

namespace trplk {

namespace {

constexpr int PQ = SYEV_MAXB;  // largest pencil
constexpr int PLD = PQ + 1;    // LDS row padding
constexpr int PT = 256;

// TA, TB (ld PQ) of the pencil with q columns; S holds the B-inner products
// of x_k with the columns of Q (S[0 .. q)) and, when up, of p_{k-1}
// (S[sp .. sp + q)).
__device__ void build_pencil(const double* __restrict__ T, int ldT, const double* __restrict__ S, int sp,
                             int q, bool up, double* sTA, double* sTB) {
  const int e = q - 1;
  for (int t = threadIdx.x; t < q * q; t += PT) {
    const int i = t % q, j = t / q;
    sTA[i * PLD + j] = 0.5 * (T[i + static_cast<int64_t>(j) * ldT] + T[j + static_cast<int64_t>(i) * ldT]);
    double b = (i == j) ? 1.0 : 0.0;
    if (i == 0) b = S[j];
    if (j == 0) b = S[i];
    if (up) {
      if (i == e) b = S[sp + j];
      if (j == e) b = S[sp + i];
      if ((i == 0 && j == e) || (i == e && j == 0)) b = 0.5 * (S[e] + S[sp]);
    }
    sTB[i * PLD + j] = b;
  }
  __syncthreads();
}

// In-place Cholesky of the leading q x q block of sL (lower triangle kept):
// false if a pivot is not above 1e-12 of the largest diagonal entry.
__device__ bool cholesky(double* sL, int q, double* red) {
  if (threadIdx.x == 0) {
    double dmax = 0.0;
    for (int i = 0; i < q; ++i) dmax = fmax(dmax, fabs(sL[i * PLD + i]));
    red[0] = dmax;
    red[1] = 1.0;
  }
  __syncthreads();
  const double dmax = red[0];
  for (int j = 0; j < q; ++j) {
    if (threadIdx.x == 0) {
      double d = sL[j * PLD + j];
      for (int k = 0; k < j; ++k) d -= sL[j * PLD + k] * sL[j * PLD + k];
      if (!(d > 1e-12 * dmax)) red[1] = 0.0;
      sL[j * PLD + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    if (red[1] == 0.0) return false;
    const double ljj = sL[j * PLD + j];
    for (int i = j + 1 + threadIdx.x; i < q; i += PT) {
      double v = sL[i * PLD + j];
      for (int k = 0; k < j; ++k) v -= sL[i * PLD + k] * sL[j * PLD + k];
      sL[i * PLD + j] = v / ljj;
    }
    __syncthreads();
  }
  return true;
}

// work: TA, TB, L, C (each PQ x PQ, ld PQ); qdev[0] = q used (0: failed),
// qdev[1] = 1 if p_{k-1} is kept
__global__ __launch_bounds__(PT) void k_pl1_reduce(const double* __restrict__ T, int ldT,
                                                   const double* __restrict__ S, int sp, int nq, int use_p,
                                                   double* __restrict__ work, int* __restrict__ qdev,
                                                   DevState* st) {
  __shared__ double sTA[PQ * PLD];
  __shared__ double sL[PQ * PLD];
  __shared__ double red[2];
  double* gTA = work;
  double* gTB = work + PQ * PQ;
  double* gL = work + 2 * PQ * PQ;
  double* gC = work + 3 * PQ * PQ;
  int q = nq;
  bool up = use_p != 0;
  build_pencil(T, ldT, S, sp, q, up, sTA, sL);
  for (int t = threadIdx.x; t < q * q; t += PT) gTB[(t / q) * PQ + t % q] = sL[(t / q) * PLD + t % q];
  __syncthreads();
  bool ok = cholesky(sL, q, red);
  if (!ok && up) {
    // drop p_{k-1}: the leading block of the same pencil
    --q;
    up = false;
    for (int t = threadIdx.x; t < q * q; t += PT) sL[(t / q) * PLD + t % q] = gTB[(t / q) * PQ + t % q];
    __syncthreads();
    ok = cholesky(sL, q, red);
  }
  if (!ok) {
    if (threadIdx.x == 0) {
      qdev[0] = 0;
      qdev[1] = 0;
      st->pl1_err = 1;
    }
    return;
  }
  // X = L^-1 TA, one column per thread (forward substitution), in place
  for (int j = threadIdx.x; j < q; j += PT) {
    for (int i = 0; i < q; ++i) {
      double v = sTA[i * PLD + j];
      for (int k = 0; k < i; ++k) v -= sL[i * PLD + k] * sTA[k * PLD + j];
      sTA[i * PLD + j] = v / sL[i * PLD + i];
    }
  }
  __syncthreads();
  // C = X L^-T, one row per thread, in place
  for (int i = threadIdx.x; i < q; i += PT) {
    for (int j = 0; j < q; ++j) {
      double v = sTA[i * PLD + j];
      for (int k = 0; k < j; ++k) v -= sTA[i * PLD + k] * sL[j * PLD + k];
      sTA[i * PLD + j] = v / sL[j * PLD + j];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < q * q; t += PT) {
    const int i = t % q, j = t / q;
    gC[j * PQ + i] = 0.5 * (sTA[i * PLD + j] + sTA[j * PLD + i]);
    gL[i * PQ + j] = (j <= i) ? sL[i * PLD + j] : 0.0;
  }
  // TA itself (the conjugate direction needs it): rebuilt, X overwrote it
  for (int t = threadIdx.x; t < q * q; t += PT) {
    const int i = t % q, j = t / q;
    gTA[i * PQ + j] = 0.5 * (T[i + static_cast<int64_t>(j) * ldT] + T[j + static_cast<int64_t>(i) * ldT]);
  }
  if (threadIdx.x == 0) {
    qdev[0] = q;
    qdev[1] = up ? 1 : 0;
  }
}

__device__ double wave_reduce(double v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// one wavefront: lane i owns coordinate i (q <= 64)
__global__ __launch_bounds__(WAVE) void k_pl1_direction(const double* __restrict__ work,
                                                        const int* __restrict__ qdev,
                                                        const double* __restrict__ theta_c,
                                                        const double* __restrict__ Yc, int ldYc, int conj,
                                                        double rho_prev, double* __restrict__ Y, int ldY,
                                                        double* __restrict__ theta, DevState* st) {
  __shared__ double w[PQ];
  const double* gTA = work;
  const double* gTB = work + PQ * PQ;
  const double* gL = work + 2 * PQ * PQ;
  const int q = qdev[0];
  const bool up = qdev[1] != 0;
  const int i = threadIdx.x;
  if (q <= 0) return;   // the reduction failed (recorded)
  const double lambda = theta_c[0];
  // w = L^-T y: back substitution, lane i holding y_i and updating it
  double yi = i < q ? Yc[i] : 0.0;
  for (int r = q - 1; r >= 0; --r) {
    if (i == r) w[r] = yi / gL[r * PQ + r];
    __syncthreads();
    if (i < r) yi -= gL[r * PQ + i] * w[r];
  }
  __syncthreads();
  const int e = q - 1;
  const double wi = i < q ? w[i] : 0.0;
  double zg = wi;
  if (i == 0 || (up && i == e)) zg = 0.0;
  double zp = zg;
  if (up) {
    if (conj) {
      // K = TA - rho_{k-1} TB; the p coefficient makes e^T K z = 0
      const double kej = i < q ? gTA[e * PQ + i] - rho_prev * gTB[e * PQ + i] : 0.0;
      const double num = wave_reduce(kej * zg);
      const double kee = gTA[e * PQ + e] - rho_prev * gTB[e * PQ + e];
      if (i == e) zp = -num / kee;
    } else if (i == e) {
      zp = wi;
    }
  }
  // projected B-norms w^T TB w and zp^T TB zp
  __shared__ double zs[PQ];
  if (i < q) zs[i] = zp;
  __syncthreads();
  double rw = 0.0, rp = 0.0;
  if (i < q) {
    for (int j = 0; j < q; ++j) {
      const double b = gTB[i * PQ + j];
      rw += b * w[j];
      rp += b * zs[j];
    }
  }
  const double nw = sqrt(wave_reduce(wi * rw));
  const double np = sqrt(wave_reduce(zp * rp));
  int err = 0;
  if (!isfinite(lambda)) err = 2;
  else if (!(nw > 0.0) || !(np > 0.0)) err = 3;
  if (err) {
    if (i == 0) st->pl1_err = err;
    return;
  }
  for (int r = i; r < SYEV_MAXB; r += WAVE) {
    Y[r] = r < q ? w[r] / nw : 0.0;
    Y[r + ldY] = r < q ? zs[r] / np : 0.0;
  }
  if (i == 0) {
    theta[0] = lambda;
    theta[1] = 0.0;
    st->nb = q;
  }
}

// ---- start block: Cholesky QR ----
//
// G = X^T B X of the k start vectors (k <= 64), symmetrised, is factored as
// R^T R (R upper triangular) and Rinv = R^-1 written for the rotation
// X <- X Rinv.  flag = 1 when a column keeps less than 1e-5 of its norm
// once the previous ones are removed (pivot^2 <= 1e-10 of its diagonal
// entry: the Gram route, applied twice, is accurate for condition numbers
// well below 1/sqrt(eps), and the caller then orthonormalises column by
// column instead) or a value is not finite.
__global__ __launch_bounds__(PT) void k_chol_inv(const double* __restrict__ G, int ldg, int k,
                                                 double* __restrict__ Rinv, int ldr, int* __restrict__ flag) {
  __shared__ double sR[PQ * PLD];   // R^T in the lower triangle (row i, column j <= i)
  __shared__ double sI[PQ * PLD];   // Rinv, column j in row j of sI (transposed)
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int t = threadIdx.x; t < k * k; t += PT) {
    const int i = t % k, j = t / k;
    sR[i * PLD + j] = 0.5 * (G[i + static_cast<int64_t>(j) * ldg] + G[j + static_cast<int64_t>(i) * ldg]);
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (threadIdx.x == 0) {
      const double g = sR[j * PLD + j];
      double d = g;
      for (int q = 0; q < j; ++q) d -= sR[j * PLD + q] * sR[j * PLD + q];
      if (!(d > 1e-10 * g) || !(g < 1.0e300)) bad = 1;
      sR[j * PLD + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double rjj = sR[j * PLD + j];
    for (int i = j + 1 + threadIdx.x; i < k; i += PT) {
      double v = sR[i * PLD + j];
      for (int q = 0; q < j; ++q) v -= sR[i * PLD + q] * sR[j * PLD + q];
      sR[i * PLD + j] = v / rjj;
    }
    __syncthreads();
  }
  // Rinv column c solves R y = e_c (back substitution, one thread per column)
  for (int c = threadIdx.x; c < k; c += PT) {
    for (int i = k - 1; i >= 0; --i) {
      double v = (i == c) ? 1.0 : 0.0;
      if (i <= c) {
        for (int q = i + 1; q <= c; ++q) v -= sR[q * PLD + i] * sI[c * PLD + q];
        v /= sR[i * PLD + i];
      } else {
        v = 0.0;
      }
      sI[c * PLD + i] = v;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k * k; t += PT) {
    const int i = t % k, c = t / k;
    const double v = sI[c * PLD + i];
    if (!isfinite(v)) bad = 1;
    Rinv[i + static_cast<int64_t>(c) * ldr] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) *flag = bad;
}

// T(0:k, 0:k) <- (T + T^T) / 2
__global__ void k_symmetrise(double* T, int ldT, int k) {
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int i = t % k, j = t / k;
    if (i < j) {
      const double v = 0.5 * (T[i + static_cast<int64_t>(j) * ldT] + T[j + static_cast<int64_t>(i) * ldT]);
      T[i + static_cast<int64_t>(j) * ldT] = v;
      T[j + static_cast<int64_t>(i) * ldT] = v;
    }
  }
}

// the solver state after a start block of k vectors: k columns, k products
// with A and, with B != I, k with B
__global__ void k_start_state(DevState* st, int k, int with_b) {
  st->nb = k;
  st->cnt_append = k;
  st->cnt_norm = with_b ? k : 0;
}

}  // namespace

int64_t pl1_work_doubles() { return 4LL * PQ * PQ + 2 * PQ + PQ * PQ; }

hipError_t pl1_pencil(const double* T, int ldT, const double* S, int sp, int nq, bool use_p, bool conj,
                      double rho_prev, double* work, int* qdev, double* Y, int ldY, double* theta,
                      DevState* st, hipStream_t s) {
  if (nq < 1 || nq > PQ) return hipErrorInvalidValue;
  double* theta_c = work + 4 * PQ * PQ;
  double* Yc = theta_c + 2 * PQ;
  hipLaunchKernelGGL(k_pl1_reduce, dim3(1), dim3(PT), 0, s, T, ldT, S, sp, nq, use_p ? 1 : 0, work, qdev,
                     st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = syev(work + 3 * PQ * PQ, PQ, 0, qdev, 0, theta_c, Yc, PQ, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pl1_direction, dim3(1), dim3(WAVE), 0, s, work, qdev, theta_c, Yc, PQ, conj ? 1 : 0,
                     rho_prev, Y, ldY, theta, st);
  return hipGetLastError();
}

hipError_t chol_inv(const double* G, int ldg, int k, double* Rinv, int ldr, int* flag, hipStream_t s) {
  if (k < 1 || k > PQ) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(PT), 0, s, G, ldg, k, Rinv, ldr, flag);
  return hipGetLastError();
}

hipError_t symmetrise(double* T, int ldT, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_symmetrise, dim3(1), dim3(256), 0, s, T, ldT, k);
  return hipGetLastError();
}

hipError_t start_state(DevState* st, int k, bool with_b, hipStream_t s) {
  hipLaunchKernelGGL(k_start_state, dim3(1), dim3(1), 0, s, st, k, with_b ? 1 : 0);
  return hipGetLastError();
}

}  // namespace trplk
