// Rayleigh-Ritz on the projected matrix: T = Y Theta Y^T (Alg. 1).
//
// T is at most 64 x 64 (the maximum basis size), so one workgroup holds T
// and the accumulated rotations in LDS and runs the cyclic two-sided Jacobi
// method with the round-robin (tournament) ordering: in each round b/2
// disjoint index pairs are rotated at once; since the rotations of a round
// commute, J^T A J splits into independent 2 x 2 blocks, so a round is one
// parameter phase and one update phase.  Sweeps
// repeat until the off-diagonal Frobenius norm falls below 1e-15 of the
// matrix norm.  The rotation angle follows the symmetric 2 x 2 Schur
// decomposition of Golub and Van Loan (Sec. 8.5.2).  Eigenvalues are
// returned in ascending order with their eigenvectors.
#include <hip/hip_runtime.h>

#include "common.h"

namespace trplk {

namespace {

constexpr int NT = 1024;  // 16 wavefronts: every 2 x 2 block of a round has its own thread
constexpr int MB = SYEV_MAXB;
constexpr int LDA = MB + 1;  // padding against LDS bank conflicts

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < NT / WAVE; ++i) t += red[i];
  return t;
}

__global__ __launch_bounds__(NT) void k_syev(const double* T, int ldT, int b_fixed,
                                             const int* nb_dev, int nb_off, double* theta,
                                             double* Y, int ldY) {
  __shared__ double A[MB * LDA];
  __shared__ double V[MB * LDA];
  __shared__ double cs[MB / 2][2];
  __shared__ int pr[MB / 2][2];
  __shared__ double red[NT / WAVE];
  int b = nb_dev ? (*nb_dev + nb_off) : b_fixed;
  if (b > MB) b = MB;
  if (b <= 0) return;
  const int be = b + (b & 1);
  const int tid = threadIdx.x;
  for (int t = tid; t < be * be; t += NT) {
    const int i = t % be, j = t / be;
    A[i * LDA + j] = (i < b && j < b) ? T[i + static_cast<int64_t>(j) * ldT] : 0.0;
    V[i * LDA + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double fro = 0.0;
  for (int t = tid; t < be * be; t += NT) {
    const double a = A[(t % be) * LDA + t / be];
    fro += a * a;
  }
  fro = block_sum(fro, red);
  const double stop = 1e-30 * fro;  // (1e-15 ||T||_F)^2
  const int half = be / 2;
  for (int sweep = 0; sweep < 40 && be > 1; ++sweep) {
    double off = 0.0;
    for (int t = tid; t < be * be; t += NT) {
      const int i = t % be, j = t / be;
      if (i != j) off += A[i * LDA + j] * A[i * LDA + j];
    }
    off = block_sum(off, red);
    if (off <= stop) break;
    for (int r = 0; r < be - 1; ++r) {
      if (tid < half) {
        // circle schedule: player be-1 meets r, the others pair up around r
        int p, q;
        if (tid == 0) {
          p = be - 1;
          q = r;
        } else {
          const int N = be - 1;
          p = (r + tid) % N;
          q = (r - tid + N) % N;
        }
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        const double apq = A[p * LDA + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double app = A[p * LDA + p], aqq = A[q * LDA + q];
          const double tau = (aqq - app) / (2.0 * apq);
          double tt;
          if (fabs(tau) > 1e150) {
            tt = 0.5 / tau;
          } else {
            tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          }
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        pr[tid][0] = p;
        pr[tid][1] = q;
        cs[tid][0] = c;
        cs[tid][1] = s;
      }
      __syncthreads();
      // All rotations of the round commute (disjoint index pairs), so
      // A <- J^T A J splits into independent 2 x 2 blocks: block (i, j) holds
      // rows {p_i, q_i} and columns {p_j, q_j}.  V <- V J updates column pairs.
      // thread (i0, j): j = tid % 32 < half, i = i0, i0 + 8, ... (no divisions)
      for (int i = tid >> 5, j = tid & 31; i < half; i += NT / 32) {
        if (j >= half) break;
        const int p = pr[i][0], q = pr[i][1], u = pr[j][0], v = pr[j][1];
        const double ci = cs[i][0], si = cs[i][1], cj = cs[j][0], sj = cs[j][1];
        const double apu = A[p * LDA + u], apv = A[p * LDA + v];
        const double aqu = A[q * LDA + u], aqv = A[q * LDA + v];
        const double bpu = ci * apu - si * aqu, bpv = ci * apv - si * aqv;
        const double bqu = si * apu + ci * aqu, bqv = si * apv + ci * aqv;
        A[p * LDA + u] = cj * bpu - sj * bpv;
        A[p * LDA + v] = sj * bpu + cj * bpv;
        A[q * LDA + u] = cj * bqu - sj * bqv;
        A[q * LDA + v] = sj * bqu + cj * bqv;
        if (i == j && si != 0.0) {  // the annihilated pair
          A[p * LDA + v] = 0.0;
          A[q * LDA + u] = 0.0;
        }
      }
      for (int j = tid >> 6, row = tid & 63; j < half; j += NT / 64) {
        if (row >= be) break;
        const int u = pr[j][0], v = pr[j][1];
        const double cj = cs[j][0], sj = cs[j][1];
        const double vu = V[row * LDA + u], vv = V[row * LDA + v];
        V[row * LDA + u] = cj * vu - sj * vv;
        V[row * LDA + v] = sj * vu + cj * vv;
      }
      __syncthreads();
    }
  }
  // ascending order; ties keep the index order
  if (tid < b) {
    const double d = A[tid * LDA + tid];
    int rank = 0;
    for (int j = 0; j < b; ++j) {
      const double e = A[j * LDA + j];
      rank += (e < d) || (e == d && j < tid);
    }
    theta[rank] = d;
    for (int i = 0; i < b; ++i) Y[i + static_cast<int64_t>(rank) * ldY] = V[i * LDA + tid];
  }
}

}  // namespace

hipError_t syev(const double* T, int ldT, int b_fixed, const int* nb_dev, int nb_offset,
                double* theta, double* Y, int ldY, hipStream_t s) {
  hipLaunchKernelGGL(k_syev, dim3(1), dim3(NT), 0, s, T, ldT, b_fixed, nb_dev, nb_offset, theta, Y,
                     ldY);
  return hipGetLastError();
}

}  // namespace trplk
