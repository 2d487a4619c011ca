// Rayleigh-Ritz on the projected matrix: T = Y Theta Y^T (Alg. 1).
//
// T is at most 64 x 64 (the maximum basis size), so one workgroup holds T
// and the accumulated rotations in LDS and runs the cyclic two-sided Jacobi
// method with the round-robin (tournament) ordering: in each round b/2
// disjoint index pairs are rotated at once; since the rotations of a round
// commute, J^T A J splits into independent 2 x 2 blocks, so a round is one
// angle phase (the first wavefront, one lane per pair) and one update phase
// (one thread per 2 x 2 block).  Sweeps repeat until the off-diagonal
// Frobenius norm falls below 1e-15 of the matrix norm.  The angle is that of
// the symmetric 2 x 2 Schur decomposition (Golub and Van Loan, Sec. 8.5.2),
// the smaller one, |phi| <= pi/4: with d = a_qq - a_pp, e = 2 a_pq and
// r = sqrt(d^2 + e^2), cos 2phi = |d| / r and sin 2phi = sign(d) e / r, so
// by the half-angle formulas c = sqrt((1 + |d| / r) / 2) (no cancellation)
// and s = sin 2phi / (2 c).  d and e are scaled by a power of two taken from
// the largest entry so that the squares neither overflow nor underflow for
// entries that matter.  Eigenvalues are returned in ascending order with
// their eigenvectors.
#include <hip/hip_runtime.h>

#include "common.h"

namespace trplk {

namespace {

constexpr int NT = 1024;  // 16 wavefronts: every 2 x 2 block of a round has its own thread
constexpr int MB = SYEV_MAXB;
constexpr int LDA = MB + 1;  // padding against LDS bank conflicts
constexpr int MH = MB / 2;   // pairs per round at most
static_assert(MH * MH <= NT, "one thread per 2 x 2 block");

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

__device__ __forceinline__ double block_max(double v, double* red) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < NT / WAVE; ++i) t = fmax(t, red[i]);
  return t;
}

// Circle schedule on be (even) players, N = be - 1: in round r player N
// meets r, and for t = 1 .. be/2 - 1 player r + t meets r - t (mod N).
// Pair t of round r, sorted.
__device__ __forceinline__ void round_pair(int r, int t, int be, int& p, int& q) {
  const int N = be - 1;
  if (t == 0) {
    p = r;
    q = N;
    return;
  }
  int a = r + t;
  if (a >= N) a -= N;
  int b = r - t;
  if (b < 0) b += N;
  p = min(a, b);
  q = max(a, b);
}

// rotation (c, s) that annihilates a_pq of the symmetric pair (a_pp, a_qq, a_pq)
__device__ __forceinline__ void pair_angle(double app, double aqq, double apq, double sc,
                                           double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (apq == 0.0) return;
  const double d = (aqq - app) * sc, e = 2.0 * apq * sc;
  const double r2 = d * d + e * e;
  if (r2 > 0.0) {  // r2 = 0: both below 1e-154 of the largest entry, nothing to rotate
    const double ir = rsqrt(r2);
    const double x = 0.5 + 0.5 * fabs(d) * ir;  // c^2, in [1/2, 1]
    c = sqrt(x);
    s = 0.5 * (d >= 0.0 ? e : -e) * ir * rsqrt(x);
  }
}

__global__ __launch_bounds__(NT) void k_syev(const double* T, int ldT, int b_fixed,
                                             const int* nb_dev, int nb_off, double* theta,
                                             double* Y, int ldY) {
  __shared__ double A[MB * LDA];
  __shared__ double V[MB * LDA];
  __shared__ double cs[MH][2];
  __shared__ int pr[MH][2];
  __shared__ double red[NT / WAVE];
  int b = nb_dev ? (*nb_dev + nb_off) : b_fixed;
  if (b > MB) b = MB;
  if (b <= 0) return;
  const int be = b + (b & 1);
  const int half = be / 2;
  const int tid = threadIdx.x;
  double amax = 0.0;
  for (int t = tid; t < be * be; t += NT) {
    const int i = t % be, j = t / be;
    const double a = (i < b && j < b) ? T[i + static_cast<int64_t>(j) * ldT] : 0.0;
    A[i * LDA + j] = a;
    V[i * LDA + j] = (i == j) ? 1.0 : 0.0;
    amax = fmax(amax, fabs(a));
  }
  amax = block_max(amax, red);
  int ex = 0;
  frexp(amax, &ex);
  // sc = 2^-ex: amax * sc in [1/2, 1) unless subnormal; the norms and angles
  // use scaled entries, so T of any magnitude behaves alike
  const double sc = ldexp(1.0, -max(ex, -1020));
  double fro = 0.0;
  for (int t = tid; t < be * be; t += NT) {
    const double a = A[(t % be) * LDA + t / be] * sc;
    fro += a * a;
  }
  fro = block_sum(fro, red);
  const double stop = 1e-30 * fro;  // (1e-15 ||T||_F)^2
  for (int sweep = 0; sweep < 40 && be > 1; ++sweep) {
    double off = 0.0;
    for (int t = tid; t < be * be; t += NT) {
      const int i = t % be, j = t / be;
      const double a = A[i * LDA + j] * sc;
      if (i != j) off += a * a;
    }
    off = block_sum(off, red);
    if (off <= stop) break;
    for (int r = 0; r < be - 1; ++r) {
      if (tid < half) {
        int p, q;
        round_pair(r, tid, be, p, q);
        double c, s;
        pair_angle(A[p * LDA + p], A[q * LDA + q], A[p * LDA + q], sc, c, s);
        pr[tid][0] = p;
        pr[tid][1] = q;
        cs[tid][0] = c;
        cs[tid][1] = s;
      }
      __syncthreads();
      // block (i, j) holds rows {p_i, q_i} and columns {p_j, q_j} of A;
      // V <- V J updates column pairs.  thread (i, j) = (tid / 32, tid % 32)
      for (int i = tid >> 5, j = tid & 31; i < half; i += NT / 32) {
        if (j >= half) break;
        const int p = pr[i][0], q = pr[i][1], u = pr[j][0], v = pr[j][1];
        const double ci = cs[i][0], si = cs[i][1], cj = cs[j][0], sj = cs[j][1];
        const double apu = A[p * LDA + u], apv = A[p * LDA + v];
        const double aqu = A[q * LDA + u], aqv = A[q * LDA + v];
        const double vpu = V[p * LDA + u], vpv = V[p * LDA + v];
        const double vqu = V[q * LDA + u], vqv = V[q * LDA + v];
        const double bpu = ci * apu - si * aqu, bpv = ci * apv - si * aqv;
        const double bqu = si * apu + ci * aqu, bqv = si * apv + ci * aqv;
        double n_pv = sj * bpu + cj * bpv, n_qu = cj * bqu - sj * bqv;
        if (i == j && si != 0.0) {  // the annihilated pair (u = p, v = q)
          n_pv = 0.0;
          n_qu = 0.0;
        }
        A[p * LDA + u] = cj * bpu - sj * bpv;
        A[p * LDA + v] = n_pv;
        A[q * LDA + u] = n_qu;
        A[q * LDA + v] = sj * bqu + cj * bqv;
        V[p * LDA + u] = cj * vpu - sj * vpv;
        V[p * LDA + v] = sj * vpu + cj * vpv;
        V[q * LDA + u] = cj * vqu - sj * vqv;
        V[q * LDA + v] = sj * vqu + cj * vqv;
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
