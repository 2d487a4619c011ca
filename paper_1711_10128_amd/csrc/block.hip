// Block Gram-Schmidt passes of block TRPL+K on the FP64 matrix cores.
//
// H = M^T V for a basis block M (n x ncols, ncols <= 128, column-major,
// leading dimension ld) and a block V of r <= 16 vectors, and V += alpha M H.
// Both are tall-skinny products whose contraction (dot) or expansion
// (update) runs over the n rows, so one pass reads M once for all r vectors
// instead of once per vector: the arithmetic per byte of M grows with r
// (2r flops per 8 bytes) while the pass stays bound by HBM.
//
// V_MFMA_F64_16X16X4F64 operand layout (A 16 x 4, B 4 x 16, D 16 x 16): lane
// l holds A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register j
// holds D[l / 16 + 4 j][l % 16].
//
// Dot: a workgroup of eight wavefronts stages 128 rows of V in LDS; wavefront
// w owns basis columns 16 w .. 16 w + 15.  For each 16-row tile a lane loads
// four consecutive rows of its column (two 16-byte loads: the four lanes of a
// column cover 128 contiguous bytes) and issues four MFMAs, K slot q of MFMA i
// being row 4 q + i, so D = V^T M over the tile accumulates in four
// registers.  Each workgroup writes its 16 x 128 partial tile; a second
// kernel sums the partials of all workgroups in a fixed order.
//
// Update: a wavefront owns a 16-row tile and computes (M H)^T for it with
// A = H^T fragments held in registers (one per 4-column K step) and B = M^T
// read as 16 consecutive rows of 4 columns; the transposed output puts 16
// consecutive rows of one vector in consecutive lanes, so the read-modify-
// write of V is as contiguous as the loads of M.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace trplk {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int BD_WAVES = 8;    // column groups of 16: ncols <= 128
constexpr int BD_TILES = 8;    // 16-row tiles per LDS round (128 rows)
constexpr int BD_ROWS = BD_TILES * 16;
constexpr int BD_MAXBLK = 256;
constexpr int BU_THREADS = 256;

__global__ __launch_bounds__(BD_WAVES * WAVE) void k_block_dot(int n, int ncols,
                                                               const double* __restrict__ M,
                                                               int64_t ld,
                                                               const double* __restrict__ V,
                                                               int64_t ldv, int r,
                                                               double* __restrict__ partial) {
  __shared__ double Vs[BD_ROWS][17];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int li = lane & 15, lg = lane >> 4;
  const int c = wv * 16 + li;
  const bool active = wv * 16 < ncols;
  const bool colok = c < ncols;
  const double* Mc = M + static_cast<int64_t>(colok ? c : 0) * ld;
  d4 D = {0.0, 0.0, 0.0, 0.0};
  const int nround = (n + BD_ROWS - 1) / BD_ROWS;
  for (int rd = blockIdx.x; rd < nround; rd += gridDim.x) {
    const int base = rd * BD_ROWS;
    for (int e = threadIdx.x; e < BD_ROWS * 16; e += BD_WAVES * WAVE) {
      const int row = e % BD_ROWS, v = e / BD_ROWS;
      Vs[row][v] = (v < r && base + row < n) ? V[static_cast<int64_t>(v) * ldv + base + row] : 0.0;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int t = 0; t < BD_TILES; ++t) {
        const int r0 = base + t * 16 + 4 * lg;
        double b[4];
        if (colok && r0 + 3 < n) {
          const d2 p0 = *reinterpret_cast<const d2*>(Mc + r0);
          const d2 p1 = *reinterpret_cast<const d2*>(Mc + r0 + 2);
          b[0] = p0.x; b[1] = p0.y; b[2] = p1.x; b[3] = p1.y;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) b[i] = (colok && r0 + i < n) ? Mc[r0 + i] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
          D = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[t * 16 + 4 * lg + i][li], b[i], D, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // D[v][c] with v = lg + 4 j, c = 16 wv + li
  double* out = partial + static_cast<int64_t>(blockIdx.x) * (BD_WAVES * 16 * 16);
  if (colok) {
#pragma unroll
    for (int j = 0; j < 4; ++j) out[c * 16 + lg + 4 * j] = D[j];
  }
}

// H[c + v * ldh] = sum over workgroups of the partial tiles (fixed order)
__global__ void k_block_dot_finish(int nblk, int ncols, int r, const double* __restrict__ partial,
                                   double* __restrict__ H, int ldh) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncols * r) return;
  const int c = e % ncols, v = e / ncols;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[static_cast<int64_t>(b) * (BD_WAVES * 256) + c * 16 + v];
  H[c + static_cast<int64_t>(v) * ldh] = s;
}

template <int KS>
__global__ __launch_bounds__(BU_THREADS) void k_block_update(int n, int ncols,
                                                             const double* __restrict__ M,
                                                             int64_t ld,
                                                             const double* __restrict__ H, int ldh,
                                                             int r, double alpha,
                                                             double* __restrict__ V, int64_t ldv) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int li = lane & 15, lg = lane >> 4;
  // A = H^T fragments: lane holds H[4 ks + lg][li] (column c = 4 ks + lg, vector li)
  double hf[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int cc = 4 * ks + lg;
    hf[ks] = (cc < ncols && li < r) ? H[cc + static_cast<int64_t>(li) * ldh] : 0.0;
  }
  const int nks = (ncols + 3) / 4;
  const int nwave = gridDim.x * (BU_THREADS / WAVE);
  const int ntile = (n + 15) / 16;
  for (int tb = blockIdx.x * (BU_THREADS / WAVE) + threadIdx.x / WAVE; tb < ntile; tb += nwave) {
    const int row = tb * 16 + li;
    const bool ok = row < n;
    double bv[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int cc = 4 * ks + lg;
      bv[ks] = (ks < nks && ok && cc < ncols) ? M[static_cast<int64_t>(cc) * ld + row] : 0.0;
    }
    d4 D = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      if (ks < nks) D = __builtin_amdgcn_mfma_f64_16x16x4f64(hf[ks], bv[ks], D, 0, 0, 0);
    // lane holds (M H)[row][v] for v = lg + 4 j
    if (ok) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int v = lg + 4 * j;
        if (v < r) {
          double* p = V + static_cast<int64_t>(v) * ldv + row;
          *p = *p + alpha * D[j];
        }
      }
    }
  }
}

__global__ void k_scale_copy(int n, double alpha, const double* __restrict__ x, double* __restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    y[i] = alpha * x[i];
}

// T(i, nb0 + j) = T(nb0 + j, i) = H(i, j) for i <= nb0 + j: column nb0 + j of
// the projected matrix from the rows of the basis up to and including itself
// (the entries between two columns of one block come from the later one)
__global__ void k_block_tcols(const double* __restrict__ H, int ldh, int nb0, int r,
                              double* __restrict__ T, int ldT) {
  for (int j = 0; j < r; ++j) {
    const int cj = nb0 + j;
    for (int i = threadIdx.x; i <= cj; i += blockDim.x) {
      const double v = H[i + static_cast<int64_t>(j) * ldh];
      T[i + static_cast<int64_t>(cj) * ldT] = v;
      T[cj + static_cast<int64_t>(i) * ldT] = v;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t scale_copy(int n, double alpha, const double* x, double* y, hipStream_t s) {
  const int g = std::max(1, std::min((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(256), 0, s, n, alpha, x, y);
  return hipGetLastError();
}

hipError_t block_tcols(const double* H, int ldh, int nb0, int r, double* T, int ldT, hipStream_t s) {
  hipLaunchKernelGGL(k_block_tcols, dim3(1), dim3(128), 0, s, H, ldh, nb0, r, T, ldT);
  return hipGetLastError();
}

int block_dot_blocks(int n) {
  const int nround = (std::max(n, 1) + BD_ROWS - 1) / BD_ROWS;
  return std::max(1, std::min(nround, BD_MAXBLK));
}

int64_t block_partial_doubles() { return static_cast<int64_t>(BD_MAXBLK) * BD_WAVES * 256; }

hipError_t block_dot(int n, int ncols, const double* M, int64_t ld, const double* V, int64_t ldv,
                     int r, double* partial, double* H, int ldh, hipStream_t s) {
  if (n < 1 || ncols < 1 || ncols > BD_WAVES * 16 || r < 1 || r > 16 || ld % 2 != 0 ||
      (reinterpret_cast<uintptr_t>(M) & 15u) != 0 || ldh < ncols)
    return hipErrorInvalidValue;
  const int nblk = block_dot_blocks(n);
  hipLaunchKernelGGL(k_block_dot, dim3(nblk), dim3(BD_WAVES * WAVE), 0, s, n, ncols, M, ld, V, ldv, r,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int tot = ncols * r;
  hipLaunchKernelGGL(k_block_dot_finish, dim3((tot + 255) / 256), dim3(256), 0, s, nblk, ncols, r,
                     partial, H, ldh);
  return hipGetLastError();
}

hipError_t block_update(int n, int ncols, const double* M, int64_t ld, const double* H, int ldh,
                        int r, double alpha, double* V, int64_t ldv, hipStream_t s) {
  if (n < 1 || ncols < 1 || ncols > 128 || r < 1 || r > 16 || ldh < ncols) return hipErrorInvalidValue;
  const int ntile = (n + 15) / 16;
  const int want = (ntile + BU_THREADS / WAVE - 1) / (BU_THREADS / WAVE);
  const int nblk = std::max(1, std::min(want, 2048));
  const int ks = (ncols + 3) / 4;
  if (ks <= 4)
    hipLaunchKernelGGL(k_block_update<4>, dim3(nblk), dim3(BU_THREADS), 0, s, n, ncols, M, ld, H, ldh, r,
                       alpha, V, ldv);
  else if (ks <= 8)
    hipLaunchKernelGGL(k_block_update<8>, dim3(nblk), dim3(BU_THREADS), 0, s, n, ncols, M, ld, H, ldh, r,
                       alpha, V, ldv);
  else if (ks <= 16)
    hipLaunchKernelGGL(k_block_update<16>, dim3(nblk), dim3(BU_THREADS), 0, s, n, ncols, M, ld, H, ldh,
                       r, alpha, V, ldv);
  else
    hipLaunchKernelGGL(k_block_update<32>, dim3(nblk), dim3(BU_THREADS), 0, s, n, ncols, M, ld, H, ldh,
                       r, alpha, V, ldv);
  return hipGetLastError();
}

}  // namespace trplk
