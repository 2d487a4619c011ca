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
// Dot: the wavefronts own 16-row tiles of the rows (grid-stride).  For a
// tile a lane loads four consecutive rows of vector l % 16 and, per group of
// 16 basis columns, four consecutive rows of column 16 g + l % 16 (two
// 16-byte loads each: the four lanes of a column or vector cover 128
// contiguous bytes), then issues four MFMAs per group, K slot q of MFMA i
// being row 4 q + i, so D_g = V^T M_g over the tile accumulates in four
// registers.  A wavefront takes at most two groups (register budget); wider
// bases split a tile's groups over 2 or 4 wavefronts.  The wavefronts of a
// workgroup add their tiles in a fixed order through LDS, each workgroup
// writes one 16 x 128 partial tile, and a second kernel sums the partials of
// all workgroups in a fixed order.  No LDS staging: both operands load
// directly in 128-byte segments.
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

constexpr int BD_THREADS = 256;  // four wavefronts
constexpr int BD_MAXCG = 8;      // column groups of 16: ncols <= 128
constexpr int BD_STRIDE = BD_MAXCG * 16 * 16;  // doubles of one workgroup's partial tile
constexpr int BD_MAXBLK = 1024;
constexpr int BD_UNROLL = 2;     // tiles whose loads a wavefront issues together
constexpr int BU_THREADS = 256;

// rows r0 .. r0 + 3 of column p (zeros past n or for an absent column)
template <bool VEC>
__device__ __forceinline__ void load4(const double* __restrict__ p, int r0, int n, bool ok,
                                      double (&o)[4]) {
  if (VEC && ok && r0 + 3 < n) {
    const d2 p0 = *reinterpret_cast<const d2*>(p + r0);
    const d2 p1 = *reinterpret_cast<const d2*>(p + r0 + 2);
    o[0] = p0.x; o[1] = p0.y; o[2] = p1.x; o[3] = p1.y;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = (ok && r0 + i < n) ? p[r0 + i] : 0.0;
  }
}

// GPW column groups per wavefront; WSPLIT wavefronts share a tile (each
// with its own groups), so a workgroup covers 4 / WSPLIT tiles at a time
// and up to GPW * WSPLIT groups.  VEC: M and V 16-byte aligned with even
// leading dimensions (two 16-byte loads per lane and operand), else scalar
// loads.
template <int GPW, int WSPLIT, bool VEC>
__global__ __launch_bounds__(BD_THREADS) void k_block_dot(int n, int ncols,
                                                          const double* __restrict__ M, int64_t ld,
                                                          const double* __restrict__ V, int64_t ldv,
                                                          int r, double* __restrict__ partial) {
  constexpr int TS = BD_THREADS / WAVE / WSPLIT;   // tile slots of the workgroup
  __shared__ double red[TS > 1 ? TS - 1 : 1][WSPLIT][GPW][4][WAVE];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int ts = wv / WSPLIT, g0 = (wv % WSPLIT) * GPW;
  const int li = lane & 15, lg = lane >> 4;
  const bool vok = li < r;
  const double* Vc = V + static_cast<int64_t>(vok ? li : 0) * ldv;
  const double* Mc[GPW];
  bool cok[GPW];
#pragma unroll
  for (int g = 0; g < GPW; ++g) {
    const int c = 16 * (g0 + g) + li;
    cok[g] = c < ncols;
    Mc[g] = M + static_cast<int64_t>(cok[g] ? c : 0) * ld;
  }
  d4 D[GPW];
#pragma unroll
  for (int g = 0; g < GPW; ++g) D[g] = d4{0.0, 0.0, 0.0, 0.0};
  const int ntile = (n + 15) / 16;
  const int nts = gridDim.x * TS;
  // tiles tl, tl + nts, ... in that order (BD_UNROLL of them loaded together)
  for (int tl = blockIdx.x * TS + ts; tl < ntile; tl += nts * BD_UNROLL) {
    double a[BD_UNROLL][4];
    double b[BD_UNROLL][GPW][4];
#pragma unroll
    for (int u = 0; u < BD_UNROLL; ++u) {
      const int tu = tl + u * nts;
      const bool in = tu < ntile;
      const int r0 = tu * 16 + 4 * lg;
      load4<VEC>(Vc, r0, n, vok && in, a[u]);
#pragma unroll
      for (int g = 0; g < GPW; ++g) load4<VEC>(Mc[g], r0, n, cok[g] && in, b[u][g]);
    }
#pragma unroll
    for (int u = 0; u < BD_UNROLL; ++u)
#pragma unroll
      for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          D[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][i], b[u][g][i], D[g], 0, 0, 0);
  }
  // the workgroup's tile of each group: tile slot 0's plus those of slots
  // 1, 2, ... in that order
  if (TS > 1) {
    if (ts > 0) {
#pragma unroll
      for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[ts - 1][wv % WSPLIT][g][j][lane] = D[g][j];
    }
    __syncthreads();
    if (ts != 0) return;
#pragma unroll
    for (int w = 0; w < TS - 1; ++w)
#pragma unroll
      for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int j = 0; j < 4; ++j) D[g][j] += red[w][wv % WSPLIT][g][j][lane];
  }
  // D_g[v][c] with v = lg + 4 j, c = 16 (g0 + g) + li
  double* out = partial + static_cast<int64_t>(blockIdx.x) * BD_STRIDE;
#pragma unroll
  for (int g = 0; g < GPW; ++g) {
    const int c = 16 * (g0 + g) + li;
    if (c < ncols) {
#pragma unroll
      for (int j = 0; j < 4; ++j) out[c * 16 + lg + 4 * j] = D[g][j];
    }
  }
}

// h = M^T v for one vector v and ncols <= NC columns: each thread takes row
// pairs (16-byte loads), the four wavefronts' sums are added in order, and
// the workgroup writes partial[b][c][0] of the dot pass's layout
template <int NC>
__global__ __launch_bounds__(BD_THREADS) void k_dot_small(int n, int ncols, const double* __restrict__ M,
                                                          int64_t ld, const double* __restrict__ v,
                                                          double* __restrict__ partial) {
  __shared__ double red[NC][BD_THREADS / WAVE];
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  const int npair = (n + 1) / 2;
  for (int pr = blockIdx.x * BD_THREADS + threadIdx.x; pr < npair; pr += gridDim.x * BD_THREADS) {
    const int row = 2 * pr;
    if (row + 1 < n) {
      const d2 x = *reinterpret_cast<const d2*>(v + row);
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c < ncols) {
          const d2 m = *reinterpret_cast<const d2*>(M + static_cast<int64_t>(c) * ld + row);
          acc[c] += m.x * x.x;
          acc[c] += m.y * x.y;
        }
    } else {
      const double x = v[row];
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c < ncols) acc[c] += M[static_cast<int64_t>(c) * ld + row] * x;
    }
  }
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double t = wave_sum(acc[c]);
    if (lane == 0) red[c][wv] = t;
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < NC && c < ncols) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < BD_THREADS / WAVE; ++w) t += red[c][w];
    partial[static_cast<int64_t>(blockIdx.x) * BD_STRIDE + c * 16] = t;
  }
}

// H[c + v * ldh] = sum over workgroups of the partial tiles: one workgroup
// per column c; thread (s, v) sums the partials of workgroups s, s + 16, ...
// in order, then the 16 slices are added in order
__global__ __launch_bounds__(256) void k_block_dot_finish(int nblk, int r,
                                                          const double* __restrict__ partial,
                                                          double* __restrict__ H, int ldh) {
  __shared__ double sl[16][16];
  const int c = blockIdx.x;
  const int v = threadIdx.x & 15, sidx = threadIdx.x >> 4;
  double acc = 0.0;
#pragma unroll 8
  for (int b = sidx; b < nblk; b += 16) acc += partial[static_cast<int64_t>(b) * BD_STRIDE + c * 16 + v];
  sl[sidx][v] = acc;
  __syncthreads();
  if (threadIdx.x < 16 && v < r) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += sl[q][v];
    H[c + static_cast<int64_t>(v) * ldh] = t;
  }
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
  const int ntile = (std::max(n, 1) + 15) / 16;
  return std::max(1, std::min(ntile, BD_MAXBLK));
}

int64_t block_partial_doubles() { return static_cast<int64_t>(BD_MAXBLK) * BD_STRIDE; }

namespace {
template <int GPW, int WSPLIT>
void launch_block_dot(bool vec, int nblk, int n, int ncols, const double* M, int64_t ld,
                      const double* V, int64_t ldv, int r, double* partial, hipStream_t s) {
  if (vec)
    hipLaunchKernelGGL((k_block_dot<GPW, WSPLIT, true>), dim3(nblk), dim3(BD_THREADS), 0, s, n, ncols, M, ld,
                       V, ldv, r, partial);
  else
    hipLaunchKernelGGL((k_block_dot<GPW, WSPLIT, false>), dim3(nblk), dim3(BD_THREADS), 0, s, n, ncols, M,
                       ld, V, ldv, r, partial);
}
}  // namespace

hipError_t block_dot(int n, int ncols, const double* M, int64_t ld, const double* V, int64_t ldv,
                     int r, double* partial, double* H, int ldh, hipStream_t s) {
  if (n < 1 || ncols < 1 || ncols > BD_MAXCG * 16 || r < 1 || r > 16 || ldh < ncols)
    return hipErrorInvalidValue;
  const bool vec = ld % 2 == 0 && ldv % 2 == 0 && (reinterpret_cast<uintptr_t>(M) & 15u) == 0 &&
                   (reinterpret_cast<uintptr_t>(V) & 15u) == 0;
  if (r == 1 && vec && ncols <= 16) {
    // one vector against a few columns (the intra-block passes and the
    // B-norm) has no matrix-core shape: a plain row-pair pass, every lane busy
    const int nblk = block_dot_blocks(n);
    if (ncols <= 1)
      hipLaunchKernelGGL(k_dot_small<1>, dim3(nblk), dim3(BD_THREADS), 0, s, n, ncols, M, ld, V, partial);
    else if (ncols <= 4)
      hipLaunchKernelGGL(k_dot_small<4>, dim3(nblk), dim3(BD_THREADS), 0, s, n, ncols, M, ld, V, partial);
    else
      hipLaunchKernelGGL(k_dot_small<16>, dim3(nblk), dim3(BD_THREADS), 0, s, n, ncols, M, ld, V, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_block_dot_finish, dim3(ncols), dim3(256), 0, s, nblk, r, partial, H, ldh);
    return hipGetLastError();
  }
  const int nblk = block_dot_blocks(n);
  const int ncg = (ncols + 15) / 16;
  // two column groups per wavefront at most (register budget: five
  // wavefronts per SIMD); wider bases split a tile's groups over 2 or 4
  // wavefronts, each loading the block's rows itself
  if (ncg == 1)
    launch_block_dot<1, 1>(vec, nblk, n, ncols, M, ld, V, ldv, r, partial, s);
  else if (ncg == 2)
    launch_block_dot<2, 1>(vec, nblk, n, ncols, M, ld, V, ldv, r, partial, s);
  else if (ncg <= 4)
    launch_block_dot<2, 2>(vec, nblk, n, ncols, M, ld, V, ldv, r, partial, s);
  else
    launch_block_dot<2, 4>(vec, nblk, n, ncols, M, ld, V, ldv, r, partial, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_block_dot_finish, dim3(ncols), dim3(256), 0, s, nblk, r, partial, H, ldh);
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
