// Factorized sparse approximate inverse (FSAI, Kolotilina and Yeremin) on
// the GPU, and the CSR transpose used to apply M = G^T G.
//
// For each row i the pattern P_i is the lower-triangular part of row i of A
// (columns <= i); with a cap, rows longer than `cap` keep the cap - 1
// off-diagonal entries of largest magnitude and the diagonal (ties: smaller
// column first).  Without a cap a row may hold at most FS = 64 lower entries.  G(i, P_i) = y /
// sqrt(y_i) with A(P_i, P_i) y = e_i, so (G A)(i, j) = 0 for j in P_i \ {i}
// and (G A G^T)(i, i) = 1.  One wavefront owns one row: it selects the
// pattern, gathers the local s x s matrix (s <= 64) into LDS with binary
// searches in the rows of A, factors it with a right-looking Cholesky and
// solves L L^T y = e_s with one back substitution (the forward solve of a unit
// vector at the last position is a single division).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "common.h"

namespace trplk {

namespace {

constexpr int FS = 64;  // max pattern size

__device__ __forceinline__ int diag_pos(const int* col, int beg, int end, int i) {
  // position of the last column <= i (columns sorted)
  int lo = beg, hi = end - 1, pos = beg - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] <= i) {
      pos = mid;
      lo = mid + 1;
    } else {
      hi = mid - 1;
    }
  }
  return pos;
}

// bad: bit 0 = a row without its diagonal entry, bit 1 = a row whose lower
// pattern is longer than the local solve holds (FS) with no cap given
__global__ void k_fsai_count(int n, const int* rowptr, const int* col, int cap, int* cnt, int* bad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int beg = rowptr[i], end = rowptr[i + 1];
    const int dp = diag_pos(col, beg, end, i);
    if (dp < beg || col[dp] != i) {
      atomicOr(bad, 1);
      cnt[i] = 0;
      continue;
    }
    const int len = dp - beg + 1;
    if (cap == 0 && len > FS) {
      atomicOr(bad, 2);
      cnt[i] = 0;
      continue;
    }
    cnt[i] = cap > 0 ? min(len, cap) : len;
  }
}

__device__ __forceinline__ double lookup(const int* rowptr, const int* col, const double* val, int r,
                                         int c) {
  int lo = rowptr[r], hi = rowptr[r + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int cm = col[mid];
    if (cm == c) return val[mid];
    if (cm < c) lo = mid + 1;
    else hi = mid - 1;
  }
  return 0.0;
}

__global__ __launch_bounds__(WAVE) void k_fsai_rows(int n, const int* rowptr, const int* col,
                                                    const double* val, int cap, const int* grow,
                                                    int* gcol, double* gval, int* bad) {
  __shared__ double S[FS * (FS + 1)];
  __shared__ int P[FS];
  const int lane = threadIdx.x;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int beg = rowptr[i], end = rowptr[i + 1];
    const int dp = diag_pos(col, beg, end, i);
    if (dp < beg || col[dp] != i) continue;  // reported by the count kernel
    const int len = dp - beg + 1;            // lower entries incl. diagonal
    if (cap == 0 && len > FS) continue;      // reported by the count kernel
    const int s = cap > 0 ? min(len, cap) : len;
    // ---- pattern ----
    if (len == s) {
      for (int a = lane; a < s; a += WAVE) P[a] = col[beg + a];
    } else {
      // keep the cap-1 largest |a_ij| (j < i), ties to the smaller column
      int outpos = 0;
      for (int e0 = 0; e0 < len - 1; e0 += WAVE) {
        const int e = e0 + lane;
        bool keep = false;
        if (e < len - 1) {
          const double ve = fabs(val[beg + e]);
          int rank = 0;
          for (int f = 0; f < len - 1; ++f) {
            const double vf = fabs(val[beg + f]);
            rank += (vf > ve) || (vf == ve && f < e);
          }
          keep = rank < cap - 1;
        }
        const unsigned long long mask = __ballot(keep);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (keep) P[outpos + before] = col[beg + e];
        outpos += __popcll(mask);
      }
      if (lane == 0) P[s - 1] = i;
    }
    __syncthreads();
    // ---- gather the lower triangle of A(P, P) ----
    for (int t = lane; t < s * s; t += WAVE) {
      const int a = t / s, b = t % s;
      if (b <= a) S[a * (FS + 1) + b] = lookup(rowptr, col, val, P[a], P[b]);
    }
    __syncthreads();
    // ---- Cholesky A(P,P) = L L^T (lower, in place) ----
    bool fail = false;
    for (int j = 0; j < s; ++j) {
      const double d = S[j * (FS + 1) + j];
      if (!(d > 0.0)) {
        fail = true;
        break;
      }
      const double ljj = sqrt(d);
      __syncthreads();
      for (int a = j + 1 + lane; a < s; a += WAVE) S[a * (FS + 1) + j] /= ljj;
      if (lane == 0) S[j * (FS + 1) + j] = ljj;
      __syncthreads();
      const int rem = s - j - 1;
      for (int t = lane; t < rem * rem; t += WAVE) {
        const int a = j + 1 + t / rem, b = j + 1 + t % rem;
        if (b <= a) S[a * (FS + 1) + b] -= S[a * (FS + 1) + j] * S[b * (FS + 1) + j];
      }
      __syncthreads();
    }
    if (fail) {
      if (lane == 0) atomicOr(bad, 1);
      continue;
    }
    // ---- L^T y = z, z = e_s / L(s-1,s-1); lane a owns y_a ----
    const double lss = S[(s - 1) * (FS + 1) + (s - 1)];
    double acc = 0.0, y = 0.0;
    for (int j = s - 1; j >= 0; --j) {
      double yj = 0.0;
      if (lane == j) {
        const double z = (j == s - 1) ? 1.0 / lss : 0.0;
        y = (z - acc) / S[j * (FS + 1) + j];
        yj = y;
      }
      yj = __shfl(yj, j, WAVE);
      if (lane < j) acc += S[j * (FS + 1) + lane] * yj;
    }
    // g = y / sqrt(y_s), sqrt(y_s) = 1 / L(s-1,s-1)
    const int o = grow[i];
    if (lane < s) {
      gcol[o + lane] = P[lane];
      gval[o + lane] = y * lss;
    }
    __syncthreads();
  }
}

__global__ void k_keys(int n, const int* rowptr, const int* col, unsigned long long* key, int* tcnt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j) {
      key[j] = (static_cast<unsigned long long>(col[j]) << 32) | static_cast<unsigned int>(i);
      atomicAdd(&tcnt[col[j]], 1);
    }
  }
}

__global__ void k_unkey(int64_t nnz, const unsigned long long* key, int* tcol) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < nnz;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x)
    tcol[t] = static_cast<int>(key[t] & 0xffffffffull);
}

int g1(int64_t n) { return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))); }

hipError_t exclusive_scan(const int* in, int* out, int n, hipStream_t s) {
  size_t tmp = 0;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in, out, n + 1, s);
  if (e != hipSuccess) return e;
  void* t = nullptr;
  e = hipMalloc(&t, std::max<size_t>(tmp, 16));
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(t, tmp, in, out, n + 1, s);
  hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(t);
  return e != hipSuccess ? e : e2;
}

}  // namespace

hipError_t exclusive_scan_i32(const int* in, int* out, int n, hipStream_t s) {
  return exclusive_scan(in, out, n, s);
}

hipError_t fsai_build(int n, const int* rowptr, const int* col, const double* val, int cap,
                      int** g_rowptr, int** g_col, double** g_val, int64_t* g_nnz, int* bad_host,
                      hipStream_t s) {
  *g_rowptr = nullptr;
  *g_col = nullptr;
  *g_val = nullptr;
  // cap = 0: the whole lower pattern of every row (rows longer than FS are
  // rejected through `bad`); otherwise at most cap <= FS entries per row
  const int ecap = cap > 0 ? std::min(cap, FS) : 0;
  int* cnt = nullptr;
  int* bad = nullptr;
  hipError_t e = hipMalloc(&cnt, sizeof(int) * (n + 1));
  if (e == hipSuccess) e = hipMalloc(&bad, sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), s);
  if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, sizeof(int) * (n + 1), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fsai_count, dim3(g1(n)), dim3(256), 0, s, n, rowptr, col, ecap, cnt, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMalloc(g_rowptr, sizeof(int) * (n + 1));
  if (e == hipSuccess) e = exclusive_scan(cnt, *g_rowptr, n, s);
  int nnz = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&nnz, *g_rowptr + n, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMalloc(g_col, sizeof(int) * std::max(nnz, 1));
  if (e == hipSuccess) e = hipMalloc(g_val, sizeof(double) * std::max(nnz, 1));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fsai_rows, dim3(std::min(n, 65536)), dim3(WAVE), 0, s, n, rowptr, col, val,
                       ecap, *g_rowptr, *g_col, *g_val, bad);
    e = hipGetLastError();
  }
  int hb = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(cnt);
  (void)hipFree(bad);
  *g_nnz = nnz;
  *bad_host = hb;
  return e;
}

hipError_t csr_transpose(int n, int64_t nnz, const int* rowptr, const int* col, const double* val,
                         int** t_rowptr, int** t_col, double** t_val, hipStream_t s) {
  *t_rowptr = nullptr;
  *t_col = nullptr;
  *t_val = nullptr;
  unsigned long long *key = nullptr, *key2 = nullptr;
  double* v2 = nullptr;
  int* tcnt = nullptr;
  hipError_t e = hipMalloc(&key, sizeof(unsigned long long) * std::max<int64_t>(nnz, 1));
  if (e == hipSuccess) e = hipMalloc(&key2, sizeof(unsigned long long) * std::max<int64_t>(nnz, 1));
  if (e == hipSuccess) e = hipMalloc(&tcnt, sizeof(int) * (n + 1));
  if (e == hipSuccess) e = hipMemsetAsync(tcnt, 0, sizeof(int) * (n + 1), s);
  if (e == hipSuccess) e = hipMalloc(t_val, sizeof(double) * std::max<int64_t>(nnz, 1));
  if (e == hipSuccess) e = hipMalloc(t_col, sizeof(int) * std::max<int64_t>(nnz, 1));
  if (e == hipSuccess) e = hipMalloc(t_rowptr, sizeof(int) * (n + 1));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_keys, dim3(g1(n)), dim3(256), 0, s, n, rowptr, col, key, tcnt);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = exclusive_scan(tcnt, *t_rowptr, n, s);
  if (e == hipSuccess && nnz > 0) {
    size_t tmp = 0;
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, key, key2, val, *t_val, static_cast<int>(nnz),
                                           0, 64, s);
    void* t = nullptr;
    if (e == hipSuccess) e = hipMalloc(&t, std::max<size_t>(tmp, 16));
    if (e == hipSuccess)
      e = hipcub::DeviceRadixSort::SortPairs(t, tmp, key, key2, val, *t_val, static_cast<int>(nnz), 0,
                                             64, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_unkey, dim3(g1(nnz)), dim3(256), 0, s, nnz, key2, *t_col);
      e = hipGetLastError();
    }
    hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    (void)hipFree(t);
  }
  (void)hipFree(key);
  (void)hipFree(key2);
  (void)hipFree(tcnt);
  (void)v2;
  return e;
}

}  // namespace trplk
