// Tall-skinny Gram-Schmidt passes over the basis, the finishing reductions
// and the small vector kernels of the inner step.
//
// The basis U is n x c (c <= 128) column-major.  Every pass streams U once
// with 16-byte loads of row pairs; when U is much larger than the caches the
// loads are non-temporal, so the streamed basis does not evict the vectors
// and the matrix that the next kernels re-read.  Rows are handled in pairs
// (2p, 2p+1); slabs that lie wholly inside the n rows load without any
// bounds test, and only the last, partial slab takes a guarded per-row path.
//
// Dot passes: one workgroup of 8 wavefronts walks slabs of row pairs;
// wavefront w owns the columns w, w+8, w+16, ... and lane j the pairs
// j, j+64, ... of the slab.  Dot products accumulate in registers across
// all slabs of the workgroup and are reduced once at the end.  The fused
// pass w <- w - U h, h2 = U^T w needs the sum over all columns of a row,
// which the wavefronts combine through a double-buffered LDS array (one
// barrier per slab), so it reads U once.
// Reductions are deterministic: fixed per-lane order, fixed shuffle tree,
// and a fixed-order sum over blocks in the finishing kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "common.h"

namespace trplk {

namespace {

constexpr int STRIDE = 3 * ORTH_MAXCOL; // partial doubles per block (up to three vectors)
constexpr int ORTH_RP = 1;              // row pairs per lane per slab: dot passes
constexpr int UPD_RP = 4;               // update-only pass
int64_t g_orth_nt_bytes = int64_t(128) << 20;  // non-temporal from this basis size

using d2 = double __attribute__((ext_vector_type(2)));

template <bool FULL, bool NT>
__device__ __forceinline__ d2 ld_pair(const double* col, int p, int n) {
  const int r = 2 * p;
  if constexpr (FULL) {
    const d2* q = reinterpret_cast<const d2*>(col + r);
    if constexpr (NT) return __builtin_nontemporal_load(q);
    else return *q;
  } else {
    d2 v;
    v.x = r < n ? col[r] : 0.0;
    v.y = r + 1 < n ? col[r + 1] : 0.0;
    return v;
  }
}

template <bool FULL>
__device__ __forceinline__ void st_pair(double* col, int p, int n, d2 v) {
  const int r = 2 * p;
  if constexpr (FULL) {
    *reinterpret_cast<d2*>(col + r) = v;
  } else {
    if (r < n) col[r] = v.x;
    if (r + 1 < n) col[r + 1] = v.y;
  }
}

template <bool FULL>
__device__ __forceinline__ void st_pair32(float* col, int p, int n, d2 v) {
  const int r = 2 * p;
  if constexpr (FULL) {
    float2 f;
    f.x = static_cast<float>(v.x);
    f.y = static_cast<float>(v.y);
    *reinterpret_cast<float2*>(col + r) = f;
  } else {
    if (r < n) col[r] = static_cast<float>(v.x);
    if (r + 1 < n) col[r + 1] = static_cast<float>(v.y);
  }
}

template <bool FULL>
__device__ __forceinline__ double pair_sq(int p, int n, d2 v) {
  const int r = 2 * p;
  if constexpr (FULL) return v.x * v.x + v.y * v.y;
  else return (r < n ? v.x * v.x : 0.0) + (r + 1 < n ? v.y * v.y : 0.0);
}

using Full = std::integral_constant<bool, true>;
using Part = std::integral_constant<bool, false>;

// Acceptance of the vector just orthogonalised, from its squared (B-)norm
// b2: a breakdown (b2 not above tol2 relative to the squared norm before
// the pass) or a non-finite value drops it; otherwise 1 / sqrt(b2) scales
// the append, and in the delayed form the appended column awaits its
// correction.
__device__ __forceinline__ void norm_accept(DevState* st, double b2, int dc, double tol2,
                                            double h1norm2) {
  st->beta2 = b2;
  st->cnt_norm += 1;
  const bool finite = (b2 == b2) && (b2 < 1.0e308);
  if (!finite) st->bad = 1;
  if (!(b2 > tol2 * (h1norm2 + b2)) || !finite) {
    st->skip = 1;  // breakdown / dropped vector: nothing is appended
  } else {
    st->inv_beta = 1.0 / sqrt(b2);
    if (dc) st->pending = 1;
  }
}

// Last-workgroup detection for a finish fused into a pass.  Each workgroup
// publishes its one partial with a device-scope atomic store (written
// through to the device-coherent level, so no writeback of the cached
// output of the pass is needed: a device-scope release fence would write
// back the whole L2 of every XCD, once per workgroup), waits for that store
// to be acknowledged, and counts itself in; the workgroup that completes the count resets the
// counter for the next pass and reads the partials with device-scope atomic
// loads.  No workgroup waits for another.
__device__ __forceinline__ void publish_partial(double* dst, double v) {
  __hip_atomic_store(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double read_partial(const double* src) {
  return __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// called by every thread after thread 0 published the workgroup's partial
__device__ __forceinline__ bool last_workgroup(int* counter) {
  __shared__ int last;
  if (threadIdx.x == 0) {
    // wait until the publishing store is acknowledged (s_waitcnt with every
    // counter at zero); the signal fences keep the compiler from moving the
    // store or the count across the wait
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const int prev = __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = prev == static_cast<int>(gridDim.x) - 1;
    if (last) __hip_atomic_store(counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return last;
}

// Squared norm of the pass output from the per-workgroup partials (stride
// STRIDE), summed in workgroup order by the last workgroup (NTH threads),
// then the acceptance decision.
template <int NTH>
__device__ __forceinline__ void norm_tail(const OrthArgs& a, double* red) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int nblk = static_cast<int>(gridDim.x);
  // the state the decision needs, loaded alongside the partials
  const DevState* st = a.state;
  const double tol2 = threadIdx.x == 0 ? st->tol2 : 0.0;
  const double h1 = threadIdx.x == 0 ? st->h1norm2 : 0.0;
  constexpr int U = 8;  // loads in flight per thread, summed in a fixed order
  double t = 0.0;
  for (int b0 = threadIdx.x; b0 < nblk; b0 += U * NTH) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * NTH;
      v[u] = b < nblk ? read_partial(a.partial + static_cast<int64_t>(b) * STRIDE) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) t += v[u];
  }
  t = wave_sum(t);
  __syncthreads();
  if (lane == 0) red[wv] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b2 = 0.0;
    for (int q = 0; q < NTH / WAVE; ++q) b2 += red[q];
    norm_accept(const_cast<DevState*>(st), b2, a.norm_dc, tol2, h1);
  }
}

// MODE ORTH_DOT: acc[i][v] = (column c of Md_v) . vec_v over the block's
// slabs.  MODE ORTH_UPD_DOT: w <- w - Mu h, then acc[i][0] = Md1(:,c) . w.
// NWV wavefronts per workgroup, wavefront w owning columns w + NWV * i.
template <int CPW, int MODE, int NV, bool SAME, int RP, bool NT, int NWV>
__global__ __launch_bounds__(NWV * WAVE) void k_orth(const OrthArgs a) {
  constexpr int SLABP = WAVE * RP;  // row pairs per slab
  if (a.state && a.state->skip) return;
  const int ncol = a.ncol_fixed + (a.state ? a.state->nb : 0) + a.ncol_extra;
  const int lane = threadIdx.x & (WAVE - 1);
  // wave-uniform: column indices, coefficients and column tests stay scalar
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int64_t ld = a.ld;
  const int n = a.n;

  double hc[CPW];
  double acc[CPW][NV];
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int c = wv + NWV * i;
    hc[i] = (MODE != ORTH_DOT && c < ncol) ? a.h[c] : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[i][v] = 0.0;
  }
  __shared__ d2 red[2][NWV][SLABP];
  // dot passes: the vectors' rows of a slab are read from memory once per
  // workgroup into LDS (double-buffered, one barrier per slab) instead of once
  // per wavefront
  __shared__ d2 vs[MODE == ORTH_DOT ? 2 : 1][NV][MODE == ORTH_DOT ? SLABP : 1];
  int buf = 0;
  const int npair = (n + 1) / 2;
  const int nslab = (npair + SLABP - 1) / SLABP;
  const int nfull = n / (2 * SLABP);  // slabs wholly inside the rows

  const double* vec0 = a.vec0;
  if (a.vec0_base) vec0 = a.vec0_base + static_cast<int64_t>(a.vec0_col0 + a.state->nb) * ld;
  const double* vec1 = a.vec1;
  if (a.vec1_base) vec1 = a.vec1_base + static_cast<int64_t>(a.vec0_col0 + a.state->nb) * ld;

  auto slab = [&](int sl, auto full) {
    constexpr bool F = decltype(full)::value;
    const int base = sl * SLABP + lane;
    if constexpr (MODE == ORTH_DOT) {
      // every load of the slab is issued before the first product.  Matrix of
      // each vector: vec0 -> Md0; two vectors: vec1 -> Md1; three vectors:
      // vec1 -> Md0, vec2 -> Md1
      constexpr int NU = (NV >= 2 && !SAME) ? 2 : 1;
      constexpr int M1 = NV == 3 ? 0 : NU - 1;
      d2 u[NU][CPW][RP];
#pragma unroll
      for (int i = 0; i < CPW; ++i) {
        const int c = wv + NWV * i;
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          u[0][i][r] = c < ncol ? ld_pair<F, NT>(a.Md0 + c * ld, base + WAVE * r, n) : d2{0.0, 0.0};
          if constexpr (NU == 2)
            u[NU - 1][i][r] =
                c < ncol ? ld_pair<F, NT>(a.Md1 + c * ld, base + WAVE * r, n) : d2{0.0, 0.0};
        }
      }
      for (int e = threadIdx.x; e < NV * SLABP; e += NWV * WAVE) {
        const int v = e / SLABP, q = e - v * SLABP;
        const double* src = v == 0 ? vec0 : v == 1 ? vec1 : a.vec2;
        vs[buf][v][q] = ld_pair<F, false>(src, sl * SLABP + q, n);
      }
      __syncthreads();
      d2 vv[NV][RP];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int r = 0; r < RP; ++r) vv[v][r] = vs[buf][v][lane + WAVE * r];
      buf ^= 1;
#pragma unroll
      for (int i = 0; i < CPW; ++i) {
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          acc[i][0] += u[0][i][r].x * vv[0][r].x;
          acc[i][0] += u[0][i][r].y * vv[0][r].y;
          if constexpr (NV >= 2) {
            acc[i][1] += u[M1][i][r].x * vv[1][r].x;
            acc[i][1] += u[M1][i][r].y * vv[1][r].y;
          }
          if constexpr (NV == 3) {
            acc[i][2] += u[NU - 1][i][r].x * vv[2][r].x;
            acc[i][2] += u[NU - 1][i][r].y * vv[2][r].y;
          }
        }
      }
    } else {
      d2 u[CPW][RP];
      d2 part[RP];
      d2 win[RP];
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        part[r] = d2{0.0, 0.0};
        win[r] = ld_pair<F, false>(a.w, base + WAVE * r, n);
      }
#pragma unroll
      for (int i = 0; i < CPW; ++i) {
        const int c = wv + NWV * i;
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          u[i][r] = c < ncol ? ld_pair<F, NT>(a.Mu + c * ld, base + WAVE * r, n) : d2{0.0, 0.0};
          part[r].x += u[i][r].x * hc[i];
          part[r].y += u[i][r].y * hc[i];
        }
      }
#pragma unroll
      for (int r = 0; r < RP; ++r) red[buf][wv][lane + WAVE * r] = part[r];
      __syncthreads();
      d2 wn[RP];
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        d2 t{0.0, 0.0};
#pragma unroll
        for (int q = 0; q < NWV; ++q) {
          const d2 x = red[buf][q][lane + WAVE * r];
          t.x += x.x;
          t.y += x.y;
        }
        wn[r].x = win[r].x - t.x;
        wn[r].y = win[r].y - t.y;
      }
      buf ^= 1;
      if (wv == 0) {
#pragma unroll
        for (int r = 0; r < RP; ++r) st_pair<F>(a.w, base + WAVE * r, n, wn[r]);
      }
#pragma unroll
      for (int i = 0; i < CPW; ++i) {
        const int c = wv + NWV * i;
        if (c < ncol) {
#pragma unroll
          for (int r = 0; r < RP; ++r) {
            const d2 ud = SAME ? u[i][r] : ld_pair<F, NT>(a.Md1 + c * ld, base + WAVE * r, n);
            acc[i][0] += ud.x * wn[r].x;
            acc[i][0] += ud.y * wn[r].y;
          }
        }
      }
    }
  };
  for (int sl = blockIdx.x; sl < nslab; sl += gridDim.x) {
    if (sl < nfull) slab(sl, Full{});
    else slab(sl, Part{});
  }

  double* out = a.partial + static_cast<int64_t>(blockIdx.x) * STRIDE;
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int c = wv + NWV * i;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double s = wave_sum(acc[i][v]);
      // three vectors: compact [v][ncol] layout (read by the delayed finish)
      if (lane == 0 && c < ncol) out[v * (NV == 3 ? ncol : ORTH_MAXCOL) + c] = s;
    }
  }
}

// Update-only pass: wout = w - U h (+ ||wout||^2).  Without dot products
// no cross-wavefront exchange is needed: every lane owns UPD_RP row pairs
// and streams all columns for them, with h staged in LDS.
constexpr int UPD_THREADS = 256;

template <bool NT>
__global__ __launch_bounds__(UPD_THREADS) void k_upd(const OrthArgs a) {
  if (a.state && a.state->skip) return;
  const int ncol = a.ncol_fixed + (a.state ? a.state->nb : 0) + a.ncol_extra;
  __shared__ double hs[ORTH_MAXCOL];
  __shared__ double red[UPD_THREADS / WAVE];
  for (int c = threadIdx.x; c < ncol; c += UPD_THREADS) hs[c] = a.h[c];
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int64_t ld = a.ld;
  const int n = a.n;
  constexpr int TILEP = WAVE * UPD_RP;
  const int npair = (n + 1) / 2;
  const int ntile = (npair + TILEP - 1) / TILEP;
  const int nfull = n / (2 * TILEP);
  double nacc = 0.0;
  auto tile_body = [&](int tile, auto full) {
    constexpr bool F = decltype(full)::value;
    const int base = tile * TILEP + lane;
    d2 part[UPD_RP];
#pragma unroll
    for (int r = 0; r < UPD_RP; ++r) part[r] = d2{0.0, 0.0};
    int c = 0;
    for (; c + 4 <= ncol; c += 4) {
      d2 u[4][UPD_RP];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < UPD_RP; ++r)
          u[q][r] = ld_pair<F, NT>(a.Mu + (c + q) * ld, base + WAVE * r, n);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < UPD_RP; ++r) {
          part[r].x += u[q][r].x * hs[c + q];
          part[r].y += u[q][r].y * hs[c + q];
        }
    }
    for (; c < ncol; ++c) {
#pragma unroll
      for (int r = 0; r < UPD_RP; ++r) {
        const d2 u = ld_pair<F, NT>(a.Mu + c * ld, base + WAVE * r, n);
        part[r].x += u.x * hs[c];
        part[r].y += u.y * hs[c];
      }
    }
#pragma unroll
    for (int r = 0; r < UPD_RP; ++r) {
      const int p = base + WAVE * r;
      const d2 w = ld_pair<F, false>(a.w, p, n);
      d2 wn;
      wn.x = w.x - part[r].x;
      wn.y = w.y - part[r].y;
      st_pair<F>(a.wout, p, n, wn);
      if (a.wout32) st_pair32<F>(a.wout32, p, n, wn);
      nacc += pair_sq<F>(p, n, wn);
    }
  };
  for (int tile = blockIdx.x * (UPD_THREADS / WAVE) + wv; tile < ntile;
       tile += gridDim.x * (UPD_THREADS / WAVE)) {
    if (tile < nfull) tile_body(tile, Full{});
    else tile_body(tile, Part{});
  }
  if (a.norm) {
    nacc = wave_sum(nacc);
    if (lane == 0) red[wv] = nacc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < UPD_THREADS / WAVE; ++q) t += red[q];
      double* dst = a.partial + static_cast<int64_t>(blockIdx.x) * STRIDE;
      if (a.fuse_norm) publish_partial(dst, t);
      else *dst = t;
    }
    if (a.fuse_norm && last_workgroup(&const_cast<DevState*>(a.state)->arrive))
      norm_tail<UPD_THREADS>(a, red);
  }
}

// Delayed step (one basis pass for two vectors).  The column j = nb - 1
// holds u', a vector orthogonalised once and scaled to unit (B-)norm; c =
// U(:, 0:j)^T B u' and inv_gamma come from the previous dot pass.  Per row:
//   u    = (u' - U(:, 0:j) c) inv_gamma      (written back to column j)
//   B u  = (B u' - BU(:, 0:j) c) inv_gamma   (GEN: B != I, Md1 = B U)
//   wout = w - U(:, 0:j) h(0:j) - u h(j)     (when w is given, + ||wout||^2
//                                             for B = I)
// Columns 0..j-1 are read once for all sums; every lane reads the rows of
// column j it writes, so the in-place update is safe.  inv_gamma == 0 means
// no column is pending (the finish found none): then j = nb and only w is
// projected.
template <bool NT, bool GEN>
__global__ __launch_bounds__(UPD_THREADS) void k_upd2(const OrthArgs a) {
  if (a.state->skip) return;
  constexpr int RPU = GEN ? 2 : UPD_RP;  // row pairs per lane (two matrices: fewer)
  constexpr int CB = 4;                  // columns per batch of loads
  const double ig = a.state->inv_gamma;
  const bool corr = ig != 0.0;
  const int j = a.ncol_fixed + a.state->nb - (corr ? 1 : 0);
  __shared__ double hs[ORTH_MAXCOL];
  __shared__ double cs[ORTH_MAXCOL];
  __shared__ double red[UPD_THREADS / WAVE];
  const bool withw = a.w != nullptr;
  for (int c = threadIdx.x; c < j; c += UPD_THREADS) {
    cs[c] = a.c[c];
    hs[c] = withw ? a.h[c] : 0.0;
  }
  __syncthreads();
  const double hl = (withw && corr) ? a.h[j] : 0.0;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int64_t ld = a.ld;
  const int n = a.n;
  double* ucol = const_cast<double*>(a.Mu) + static_cast<int64_t>(j) * ld;
  double* bcol = GEN ? const_cast<double*>(a.Md1) + static_cast<int64_t>(j) * ld : nullptr;
  constexpr int TILEP = WAVE * RPU;
  const int npair = (n + 1) / 2;
  const int ntile = (npair + TILEP - 1) / TILEP;
  const int nfull = n / (2 * TILEP);
  double nacc = 0.0;
  auto tile_body = [&](int tile, auto full) {
    constexpr bool F = decltype(full)::value;
    const int base = tile * TILEP + lane;
    d2 pu[RPU], pw[RPU], pb[RPU];
#pragma unroll
    for (int r = 0; r < RPU; ++r) {
      pu[r] = d2{0.0, 0.0};
      pw[r] = d2{0.0, 0.0};
      pb[r] = d2{0.0, 0.0};
    }
    // the rows of u' and w this lane rewrites, loaded before the basis
    // stream so that their latency is not exposed at the end of the tile
    // (+1.6% on the 256^3 operator despite three wavefronts per SIMD instead
    // of four)
    d2 upre[RPU], wpre[RPU];
#pragma unroll
    for (int r = 0; r < RPU; ++r) {
      const int p = base + WAVE * r;
      upre[r] = corr ? ld_pair<F, false>(ucol, p, n) : d2{0.0, 0.0};
      wpre[r] = withw ? ld_pair<F, false>(a.w, p, n) : d2{0.0, 0.0};
    }
    int c = 0;
    for (; c + CB <= j; c += CB) {
      d2 u[CB][RPU], bq[GEN ? CB : 1][RPU];
#pragma unroll
      for (int q = 0; q < CB; ++q)
#pragma unroll
        for (int r = 0; r < RPU; ++r) {
          u[q][r] = ld_pair<F, NT>(a.Mu + (c + q) * ld, base + WAVE * r, n);
          if constexpr (GEN) bq[q][r] = ld_pair<F, NT>(a.Md1 + (c + q) * ld, base + WAVE * r, n);
        }
#pragma unroll
      for (int q = 0; q < CB; ++q)
#pragma unroll
        for (int r = 0; r < RPU; ++r) {
          pu[r].x += u[q][r].x * cs[c + q];
          pu[r].y += u[q][r].y * cs[c + q];
          pw[r].x += u[q][r].x * hs[c + q];
          pw[r].y += u[q][r].y * hs[c + q];
          if constexpr (GEN) {
            pb[r].x += bq[GEN ? q : 0][r].x * cs[c + q];
            pb[r].y += bq[GEN ? q : 0][r].y * cs[c + q];
          }
        }
    }
    for (; c < j; ++c) {
#pragma unroll
      for (int r = 0; r < RPU; ++r) {
        const d2 u = ld_pair<F, NT>(a.Mu + c * ld, base + WAVE * r, n);
        pu[r].x += u.x * cs[c];
        pu[r].y += u.y * cs[c];
        pw[r].x += u.x * hs[c];
        pw[r].y += u.y * hs[c];
        if constexpr (GEN) {
          const d2 bu = ld_pair<F, NT>(a.Md1 + c * ld, base + WAVE * r, n);
          pb[r].x += bu.x * cs[c];
          pb[r].y += bu.y * cs[c];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RPU; ++r) {
      const int p = base + WAVE * r;
      d2 un{0.0, 0.0};
      if (corr) {
        const d2 up = upre[r];
        un.x = (up.x - pu[r].x) * ig;
        un.y = (up.y - pu[r].y) * ig;
        st_pair<F>(ucol, p, n, un);
        if constexpr (GEN) {
          const d2 bp = ld_pair<F, false>(bcol, p, n);
          d2 bn;
          bn.x = (bp.x - pb[r].x) * ig;
          bn.y = (bp.y - pb[r].y) * ig;
          st_pair<F>(bcol, p, n, bn);
        }
      }
      if (withw) {
        const d2 w = wpre[r];
        d2 wn;
        wn.x = w.x - pw[r].x - un.x * hl;
        wn.y = w.y - pw[r].y - un.y * hl;
        st_pair<F>(a.wout, p, n, wn);
        if (a.wout32) st_pair32<F>(a.wout32, p, n, wn);
        nacc += pair_sq<F>(p, n, wn);
      }
    }
  };
  for (int tile = blockIdx.x * (UPD_THREADS / WAVE) + wv; tile < ntile;
       tile += gridDim.x * (UPD_THREADS / WAVE)) {
    if (tile < nfull) tile_body(tile, Full{});
    else tile_body(tile, Part{});
  }
  if (a.norm) {
    nacc = wave_sum(nacc);
    if (lane == 0) red[wv] = nacc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < UPD_THREADS / WAVE; ++q) t += red[q];
      double* dst = a.partial + static_cast<int64_t>(blockIdx.x) * STRIDE;
      if (a.fuse_norm) publish_partial(dst, t);
      else *dst = t;
    }
    if (a.fuse_norm && last_workgroup(&const_cast<DevState*>(a.state)->arrive))
      norm_tail<UPD_THREADS>(a, red);
  }
}

template <int CPW, int RP, bool NT, int NWV>
hipError_t launch_rp(int mode, const OrthArgs& a, int nblk, hipStream_t s) {
  const dim3 g(nblk), b(NWV * WAVE);
  const bool same = (mode == ORTH_DOT) ? (a.nvec == 1 || a.Md0 == a.Md1) : (a.Mu == a.Md1);
  if (mode == ORTH_DOT) {
    if (a.nvec == 1) {
      hipLaunchKernelGGL((k_orth<CPW, ORTH_DOT, 1, true, RP, NT, NWV>), g, b, 0, s, a);
    } else if (same) {
      hipLaunchKernelGGL((k_orth<CPW, ORTH_DOT, 2, true, RP, NT, NWV>), g, b, 0, s, a);
    } else {
      hipLaunchKernelGGL((k_orth<CPW, ORTH_DOT, 2, false, RP, NT, NWV>), g, b, 0, s, a);
    }
  } else {
    if (same) hipLaunchKernelGGL((k_orth<CPW, ORTH_UPD_DOT, 1, true, RP, NT, NWV>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_orth<CPW, ORTH_UPD_DOT, 1, false, RP, NT, NWV>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

template <int CPW, bool NT, int NWV>
hipError_t launch_cpw(int mode, const OrthArgs& a, int nblk, hipStream_t s) {
  return launch_rp<CPW, ORTH_RP, NT, NWV>(mode, a, nblk, s);
}

template <bool NT>
hipError_t launch_width(int mode, const OrthArgs& a, int need, int nblk, hipStream_t s) {
  if (mode == ORTH_DOT) {
    // dot passes: 16 wavefronts per workgroup on half the workgroups (half
    // the partial rows for the finishing reduction, the vectors staged once
    // for 16 wavefronts)
    const int cpw16 = (std::max(need, 1) + 15) / 16;
    if (cpw16 <= 1) return launch_cpw<1, NT, 16>(mode, a, nblk, s);
    if (cpw16 <= 2) return launch_cpw<2, NT, 16>(mode, a, nblk, s);
    if (cpw16 <= 4) return launch_cpw<4, NT, 16>(mode, a, nblk, s);
    return launch_cpw<8, NT, 16>(mode, a, nblk, s);
  }
  // fused update + dot: 8 wavefronts owning ceil(need / 8) columns each (16
  // wavefronts measured slower on MI355X: the per-slab LDS exchange and
  // barrier over 16 wavefronts cost more than the occupancy gains)
  const int cpw = (std::max(need, 1) + 7) / 8;
  if (cpw > 8) return launch_cpw<16, NT, 8>(mode, a, nblk, s);
  if (cpw <= 1) return launch_cpw<1, NT, 8>(mode, a, nblk, s);
  if (cpw <= 2) return launch_cpw<2, NT, 8>(mode, a, nblk, s);
  if (cpw <= 4) return launch_cpw<4, NT, 8>(mode, a, nblk, s);
  return launch_cpw<8, NT, 8>(mode, a, nblk, s);
}

// ------------------------------------------------------------- finish --
// One workgroup of 16 wavefronts sums the per-block partials.  Output column
// j of a sum is owned by lane j % 64: wavefront w adds blocks w, w+16, ...
// (coalesced across lanes) with FIN_UNR independent loads in flight per lane
// (summed in a fixed order), then the 16 wavefront sums are added in a fixed
// order.  fin_sum2 reduces two column ranges of up to 64 columns in the same
// pass (the T column and the first Gram-Schmidt coefficients).
constexpr int FIN_THREADS = 1024;
constexpr int FIN_WAVES = FIN_THREADS / WAVE;
constexpr int FIN_UNR = 16;

// Sum over the blocks of partial[b * stride + src + idx] for one lane; 0 if
// the lane has no column.
__device__ __forceinline__ double fin_lane(const FinishArgs& f, int src, int idx, bool on) {
  const int lane_w = threadIdx.x / WAVE;
  const double* p = f.partial + src + idx;
  const int64_t st = f.stride;
  double t[FIN_UNR];
#pragma unroll
  for (int u = 0; u < FIN_UNR; ++u) t[u] = 0.0;
  if (on) {
    int b = lane_w;
    for (; b + (FIN_UNR - 1) * FIN_WAVES < f.nblk; b += FIN_UNR * FIN_WAVES) {
#pragma unroll
      for (int u = 0; u < FIN_UNR; ++u) t[u] += p[(b + u * FIN_WAVES) * st];
    }
#pragma unroll
    for (int u = 0; u < FIN_UNR; ++u)
      if (b + u * FIN_WAVES < f.nblk) t[u] += p[(b + u * FIN_WAVES) * st];
  }
  // fixed pairwise order
#pragma unroll
  for (int w = FIN_UNR / 2; w >= 1; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) t[u] += t[u + w];
  return t[0];
}

__device__ void fin_sum(const FinishArgs& f, int src, int cnt, double* dst, double (*red)[WAVE]) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  for (int c0 = 0; c0 < cnt; c0 += WAVE) {
    const int idx = c0 + lane;
    const double t = fin_lane(f, src, idx, idx < cnt);
    red[wv][lane] = t;
    __syncthreads();
    if (wv == 0 && idx < cnt) {
      double u = 0.0;
      for (int q = 0; q < FIN_WAVES; ++q) u += red[q][lane];
      dst[idx] = u;
    }
    __syncthreads();
  }
}

// Two ranges at once (each at most 64 columns): waves 0..7 take range A,
// waves 8..15 range B, each half summing every 8th block.
__device__ void fin_sum2(const FinishArgs& f, int srcA, int cntA, double* dstA, int srcB, int cntB,
                         double* dstB, double (*red)[WAVE]) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  constexpr int HALF = FIN_WAVES / 2;
  const bool isA = wv < HALF;
  const int src = isA ? srcA : srcB;
  const int cnt = isA ? cntA : cntB;
  const double* p = f.partial + src + lane;
  const int64_t st = f.stride;
  double t[FIN_UNR];
#pragma unroll
  for (int u = 0; u < FIN_UNR; ++u) t[u] = 0.0;
  if (lane < cnt) {
    int b = wv % HALF;
    for (; b + (FIN_UNR - 1) * HALF < f.nblk; b += FIN_UNR * HALF) {
#pragma unroll
      for (int u = 0; u < FIN_UNR; ++u) t[u] += p[(b + u * HALF) * st];
    }
#pragma unroll
    for (int u = 0; u < FIN_UNR; ++u)
      if (b + u * HALF < f.nblk) t[u] += p[(b + u * HALF) * st];
  }
#pragma unroll
  for (int w = FIN_UNR / 2; w >= 1; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) t[u] += t[u + w];
  red[wv][lane] = t[0];
  __syncthreads();
  if ((wv == 0 || wv == HALF) && lane < cnt) {
    double u = 0.0;
    for (int q = 0; q < HALF; ++q) u += red[wv + q][lane];
    (isA ? dstA : dstB)[lane] = u;
  }
  __syncthreads();
}

// sum of v[c]^2, c < cnt (<= 2 * 64), by the first wavefront: lane j takes
// c = j and j + 64, then a fixed shuffle tree
__device__ __forceinline__ double sumsq_wave(const double* v, int cnt) {
  const int lane = threadIdx.x & (WAVE - 1);
  double t = 0.0;
  for (int c = lane; c < cnt; c += WAVE) t += v[c] * v[c];
  return wave_sum(t);
}

// One column summed over the blocks by all 1024 threads.
__device__ double fin_one(const FinishArgs& f, int src, double (*red)[WAVE]) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  double t = 0.0;
  for (int b = threadIdx.x; b < f.nblk; b += FIN_THREADS) t += f.partial[b * static_cast<int64_t>(f.stride) + src];
  t = wave_sum(t);
  if (lane == 0) red[0][wv] = t;
  __syncthreads();
  double u = 0.0;
  for (int q = 0; q < FIN_WAVES; ++q) u += red[0][q];
  __syncthreads();
  return u;
}

__global__ __launch_bounds__(FIN_THREADS) void k_finish(const FinishArgs f) {
  DevState* st = f.state;
  if (st && st->skip) return;
  const int nb = st ? st->nb : 0;
  __shared__ double red[FIN_WAVES][WAVE];
  __shared__ double v0[2 * ORTH_MAXCOL];
  __shared__ double v1[ORTH_MAXCOL];
  const int tid = threadIdx.x;
  switch (f.mode) {
    case FIN_TH:
    case FIN_T: {
      // new column j = nb of T; the dots cover U columns 0..nb (after the
      // ncol_fixed locked columns)
      const int j = nb;
      const int nc = f.ncol_fixed + nb + 1;
      if (f.mode == FIN_TH && j + 1 <= WAVE && nc <= WAVE) {
        fin_sum2(f, f.ncol_fixed, j + 1, v0, ORTH_MAXCOL, nc, v1, red);
      } else {
        fin_sum(f, f.ncol_fixed, j + 1, v0, red);
        if (f.mode == FIN_TH) fin_sum(f, ORTH_MAXCOL, nc, v1, red);
      }
      for (int r = tid; r <= j; r += blockDim.x) {
        f.T[r + static_cast<int64_t>(j) * f.ldT] = v0[r];
        f.T[j + static_cast<int64_t>(r) * f.ldT] = v0[r];
      }
      if (f.mode == FIN_TH) {
        if (f.skip_first) {
          if (tid == 0) v1[f.ncol_fixed] = 0.0;
          __syncthreads();
        }
        for (int c = tid; c < nc; c += blockDim.x) f.h[c] = v1[c];
        if (tid < WAVE) {
          const double t = sumsq_wave(v1, nc);
          if (tid == 0) st->h1norm2 = t;
        }
      }
      __syncthreads();
      if (tid == 0) {
        st->nb = nb + 1;
        st->cnt_append += 1;
      }
      break;
    }
    case FIN_TCOL: {
      const int j = f.cnt;
      fin_sum(f, 0, j + 1, v0, red);
      for (int r = tid; r <= j; r += blockDim.x) {
        f.T[r + static_cast<int64_t>(j) * f.ldT] = v0[r];
        f.T[j + static_cast<int64_t>(r) * f.ldT] = v0[r];
      }
      break;
    }
    case FIN_RES: {
      fin_sum(f, 0, 128, v0, red);
      for (int i = tid; i < f.cnt; i += blockDim.x) {
        const double r2 = v0[i], x2 = v0[64 + i];
        f.out[i] = sqrt(r2 / x2);
        f.out[64 + i] = sqrt(x2);
      }
      break;
    }
    case FIN_H:
    case FIN_H2: {
      const int nc = f.ncol_fixed + nb + f.extra;
      fin_sum(f, 0, nc, v0, red);
      if (f.skip_first) {
        if (tid == 0) v0[f.ncol_fixed] = 0.0;
        __syncthreads();
      }
      for (int c = tid; c < nc; c += blockDim.x) f.h[c] = v0[c];
      if (f.mode == FIN_H && tid < WAVE) {
        const double t = sumsq_wave(v0, nc);
        if (tid == 0) st->h1norm2 = t;
      }
      break;
    }
    case FIN_NORM: {
      const double b2 = fin_one(f, 0, red);
      if (tid == 0) norm_accept(st, b2, f.dc, st->tol2, st->h1norm2);
      break;
    }
    default: {
      for (int c0 = 0; c0 < f.cnt; c0 += 2 * ORTH_MAXCOL) {
        const int cnt = min(2 * ORTH_MAXCOL, f.cnt - c0);
        fin_sum(f, c0, cnt, v0, red);
        for (int c = tid; c < cnt; c += blockDim.x) f.out[c0 + c] = v0[c];
        __syncthreads();
      }
      break;
    }
  }
}

// Finish of the delayed step (FIN_DC).  The pending column is j = nb of the
// active basis, J = F + j in [Q U] (F locked columns): u' at U(:, j),
// z' = A u' at AU(:, j); the three-vector dot pass left, per block,
// a = [Q U](:, 0:J+1)^T B u', t = [Q U]^T z' and b = (B [Q U])^T w packed as
// [a | t | b] (J + 1 <= 128 entries each).  With c = a(0:J) and
// gamma^2 = a_J - |c|^2 the corrected column is u = (u' - [Q U] c) / gamma;
// A u = (z' - A [Q U] c) / gamma gives, with T = U^T A U and A symmetric,
//   T(i, j) = (t_{F+i} - (T c_U)_i) / gamma                 (i < j)
//   T(j, j) = (t_J - 2 c.t + c_U.(T c_U)) / gamma^2
// where c_U = c(F:J); the terms with U^T A Q c_Q and c_Q^T Q^T A Q c_Q are
// left out: Q holds converged eigenvectors (U^T A Q ~ residual size) and
// c_Q is the loss of orthogonality of one Gram-Schmidt pass, so they are
// far below rounding of T.  The new direction's coefficients are
// h(0:J) = b(0:J), h(J) = (b_J - c.b) / gamma (nvec = 3; nvec = 2 ignores
// b).  A U(:, j) keeps the stored z': the true products are AU_stored L
// with L(:, j) = (e_j - L c_U) / gamma.
// The block sums: lane l of wavefront w loads entries 2l, 2l + 1 (+ 128 q,
// q < SLOTS) of blocks w, w + 16, ... with 16-byte loads, so one load covers
// a block's three sums when 3 (J + 1) <= 128.  The row width loaded is the
// host's bound f.cnt on 3 (J + 1), so the loads need not wait for the
// state; entries past 3 (J + 1) are summed but never used.
constexpr int DC_MAXE = 3 * ORTH_MAXCOL;  // packed entries per block row
template <int SLOTS>
__device__ __forceinline__ void dc_block_sums(const FinishArgs& f, double (*red)[DC_MAXE]) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  constexpr int U = SLOTS == 1 ? 16 : SLOTS == 2 ? 8 : 4;  // blocks in flight per lane
  d2 t[SLOTS][U];
#pragma unroll
  for (int q = 0; q < SLOTS; ++q)
#pragma unroll
    for (int u = 0; u < U; ++u) t[q][u] = d2{0.0, 0.0};
  const int64_t st = f.stride;
  const int width = min(f.cnt, DC_MAXE);
  bool on[SLOTS];
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) on[q] = 2 * lane + 2 * WAVE * q < width;
  int b = wv;
  auto ld = [&](int blk, int q) -> d2 {
    return *reinterpret_cast<const d2*>(f.partial + blk * st + 2 * lane + 2 * WAVE * q);
  };
  for (; b + (U - 1) * FIN_WAVES < f.nblk; b += U * FIN_WAVES) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < SLOTS; ++q)
        if (on[q]) t[q][u] += ld(b + u * FIN_WAVES, q);
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (b + u * FIN_WAVES < f.nblk)
#pragma unroll
      for (int q = 0; q < SLOTS; ++q)
        if (on[q]) t[q][u] += ld(b + u * FIN_WAVES, q);
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) {
#pragma unroll
    for (int w = U / 2; w >= 1; w >>= 1)
#pragma unroll
      for (int u = 0; u < w; ++u) t[q][u] += t[q][u + w];
    const int e = 2 * lane + 2 * WAVE * q;
    red[wv][e] = t[q][0].x;
    red[wv][e + 1] = t[q][0].y;
  }
}

__global__ __launch_bounds__(FIN_THREADS) void k_finish_dc(const FinishArgs f) {
  DevState* st = f.state;
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1), wv = tid / WAVE;
  __shared__ double red[FIN_WAVES][DC_MAXE];
  __shared__ double s3[DC_MAXE];
  if (f.cnt <= 2 * WAVE) dc_block_sums<1>(f, red);
  else if (f.cnt <= 4 * WAVE) dc_block_sums<2>(f, red);
  else dc_block_sums<3>(f, red);
  // T(0:j, 0:j) and L(0:j, 0:j) entries for T c_U and L c_U: lane i owns
  // row i, wavefront w the columns w, w + 16, ... (j <= 63).  Loaded over
  // the whole 64 x 64 array before the state is known, masked below.
  constexpr int KQ = (WAVE + FIN_WAVES - 1) / FIN_WAVES;
  double tv[KQ], lv[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int k = wv + FIN_WAVES * q;
    tv[q] = f.T[lane + static_cast<int64_t>(k) * f.ldT];
    lv[q] = f.L[lane + static_cast<int64_t>(k) * f.ldT];
  }
  if (st->skip) return;
  const int F = f.ncol_fixed;
  const int j = st->nb;
  const int J = F + j;
  const int cnt = J + 1;
  const int tot = 3 * cnt;
  const bool withw = f.nvec == 3;
  // f.dc: column j is corrected only when it is pending (after a breakdown
  // nothing is: then only w is projected, against the J final columns)
  const bool corr = !f.dc || st->pending;
  if (!corr) {
    __syncthreads();
    for (int e = tid; e < J; e += FIN_THREADS) {
      double u = 0.0;
      for (int q = 0; q < FIN_WAVES; ++q) u += red[q][2 * cnt + e];
      s3[e] = u;
      if (withw) f.h[e] = u;
    }
    __syncthreads();
    if (tid < WAVE) {
      double hh = 0.0;
      for (int k = tid; k < J; k += WAVE) hh += s3[k] * s3[k];
      hh = wave_sum(hh);
      if (tid == 0) {
        st->h1norm2 = hh;
        st->inv_gamma = 0.0;  // tells the update pass: no column to correct
      }
    }
    return;
  }
  __syncthreads();
  for (int e = tid; e < tot; e += FIN_THREADS) {
    double u = 0.0;
    for (int q = 0; q < FIN_WAVES; ++q) u += red[q][e];
    s3[e] = u;
  }
  __syncthreads();
  const double* a_ = s3;
  const double* t_ = s3 + cnt;
  const double* b_ = s3 + 2 * cnt;
  const double* cu = a_ + F;  // c_U
  {
    double y = 0.0, l = 0.0;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int k = wv + FIN_WAVES * q;
      if (lane < j && k < j) {
        y += tv[q] * cu[k];
        l += lv[q] * cu[k];
      }
    }
    red[wv][lane] = y;
    red[wv][WAVE + lane] = l;
  }
  __syncthreads();
  if (wv != 0) return;
  // the first wavefront finishes alone: lane i holds (T c_U)_i and (L c_U)_i,
  // and every lane gets each dot product from the shuffle reduction
  double ys = 0.0, ls = 0.0;
  if (lane < j) {
    for (int q = 0; q < FIN_WAVES; ++q) {
      ys += red[q][lane];
      ls += red[q][WAVE + lane];
    }
  }
  double cc = 0.0, ct = 0.0, cb = 0.0, bb = 0.0;
  for (int k = lane; k < J; k += WAVE) {
    cc += a_[k] * a_[k];
    ct += a_[k] * t_[k];
    if (withw) {
      cb += a_[k] * b_[k];
      bb += b_[k] * b_[k];
    }
  }
  double cy = lane < j ? cu[lane] * ys : 0.0;
  cc = wave_sum(cc);
  ct = wave_sum(ct);
  cy = wave_sum(cy);
  cb = wave_sum(cb);
  bb = wave_sum(bb);
  const double g2 = a_[J] - cc;
  const bool ok = (g2 > 0.0) && (g2 < 1.0e308);
  const double ig = ok ? 1.0 / sqrt(g2) : 0.0;
  if (lane < j) {
    const double tij = (t_[F + lane] - ys) * ig;
    f.T[lane + static_cast<int64_t>(j) * f.ldT] = tij;
    f.T[j + static_cast<int64_t>(lane) * f.ldT] = tij;
    f.L[lane + static_cast<int64_t>(j) * f.ldT] = -ls * ig;
  }
  for (int e = lane; e < J; e += WAVE) {
    f.cbuf[e] = a_[e];
    if (withw) f.h[e] = b_[e];
  }
  if (lane == 0) {
    if (!ok) {
      st->bad = 1;
      st->skip = 1;
    }
    st->inv_gamma = ig;
    f.T[j + static_cast<int64_t>(j) * f.ldT] = (t_[J] - 2.0 * ct + cy) * ig * ig;
    f.L[j + static_cast<int64_t>(j) * f.ldT] = ig;
    if (withw) {
      const double hj = (b_[J] - cb) * ig;
      f.h[J] = hj;
      st->h1norm2 = bb + hj * hj;
    }
    st->nb = j + 1;
    st->cnt_append += 1;
    st->pending = 0;
  }
}

__global__ void k_set_state(DevState* st, int which, double dv, int iv) {
  switch (which) {
    case SET_RHO: st->rho = dv; break;
    case SET_TOL2: st->tol2 = dv; break;
    case SET_NB: st->nb = iv; break;
    case SET_SKIP: st->skip = iv; break;
    case SET_RESET_STAGE:
      st->skip = 0;
      st->tol2 = dv;
      break;
  }
}

__global__ void k_set_rho_from(DevState* st, const double* theta, int idx) { st->rho = theta[idx]; }

__global__ void k_reset_T(double* T, int ldT, int m, int kact, const double* theta, int off) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m * m; t += gridDim.x * blockDim.x) {
    const int i = t % m, j = t / m;
    T[i + static_cast<int64_t>(j) * ldT] = (i == j && i < kact) ? theta[off + i] : 0.0;
  }
}

// YA = L Y over the b = st->nb basis columns (L upper triangular); every
// column of Y is transformed (the rotation reads the first kout).
__global__ __launch_bounds__(64) void k_ly(const double* L, const double* Y, double* YA, int ld,
                                           const DevState* st) {
  // block c computes column c; thread i row i (b <= 64)
  const int b = st->nb;
  const int c = blockIdx.x, i = threadIdx.x;
  if (c >= b) return;
  __shared__ double yc[64];
  yc[i] = i < b ? Y[i + static_cast<int64_t>(c) * ld] : 0.0;
  __syncthreads();
  if (i >= b) return;
  double v = 0.0;
#pragma unroll 8
  for (int k = 0; k < b; ++k) v += L[i + static_cast<int64_t>(k) * ld] * yc[k];
  YA[i + static_cast<int64_t>(c) * ld] = v;
}

__global__ void k_eye(double* L, int ld, int m) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m * m; t += gridDim.x * blockDim.x) {
    const int i = t % m, j = t / m;
    L[i + static_cast<int64_t>(j) * ld] = i == j ? 1.0 : 0.0;
  }
}

__global__ void k_restart_residual(int n, const double* AXt, const double* BXt, const double* theta,
                                   int t, int next, const double* dinv, double* wout, double* vout,
                                   float* vout32) {
  const double th = theta[t];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double v = AXt[i] - th * BXt[i];
    if (next == NEXT_IDENT) wout[i] = v;
    else if (next == NEXT_JACOBI) wout[i] = dinv[i] * v;
    else if (vout32) vout32[i] = static_cast<float>(v);
    else vout[i] = v;
  }
}

__global__ void k_copy_cols(int n, const double* src, int64_t lds, double* dst, int64_t ldd,
                            int ncols) {
  const int64_t total = static_cast<int64_t>(n) * ncols;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t c = t / n;
    const int64_t i = t - c * n;
    dst[c * ldd + i] = src[c * lds + i];
  }
}

__global__ void k_cast_f32(int64_t n, const double* x, float* y) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = static_cast<float>(x[i]);
}

__global__ void k_cast_f64(int64_t n, const float* x, double* y) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = static_cast<double>(x[i]);
}

__global__ void k_diag_inv(int n, const int* rowptr, const int* col, const double* val,
                           double* dinv, int* bad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double d = 0.0;
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j)
      if (col[j] == i) d = val[j];
    if (!(d > 0.0)) {
      *bad = 1;
      dinv[i] = 1.0;
    } else {
      dinv[i] = 1.0 / d;
    }
  }
}

__global__ __launch_bounds__(256) void k_row_norms(int n, const int* rowptr, const double* val,
                                                   double* pinf, double* pfro) {
  double mx = 0.0, fr = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j) {
      s += fabs(val[j]);
      fr += val[j] * val[j];
    }
    mx = fmax(mx, s);
  }
  __shared__ double smx[256], sfr[256];
  smx[threadIdx.x] = mx;
  sfr[threadIdx.x] = fr;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + o]);
      sfr[threadIdx.x] += sfr[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pinf[blockIdx.x] = smx[0];
    pfro[blockIdx.x] = sfr[0];
  }
}

int grid1d(int64_t n) { return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))); }

}  // namespace

int g_orth_maxblk = 0;  // 0: by pass

int orth_blocks(int n, int mode) {
  const int npair = (std::max(n, 1) + 1) / 2;
  if (mode == ORTH_UPD || mode == ORTH_UPD2) {
    const int tiles = (npair + WAVE * UPD_RP - 1) / (WAVE * UPD_RP);
    const int want = (tiles + UPD_THREADS / WAVE - 1) / (UPD_THREADS / WAVE);
    return std::max(1, std::min(want, g_orth_maxblk > 0 ? g_orth_maxblk : 1024));
  }
  const int nslab = (npair + WAVE * ORTH_RP - 1) / (WAVE * ORTH_RP);
  const int cap = g_orth_maxblk > 0 ? g_orth_maxblk : (mode == ORTH_DOT ? 256 : 512);
  return std::max(1, std::min(nslab, cap));
}

// largest grid of any pass: sizes the partial buffer
int orth_blocks_max(int n) {
  return std::max({orth_blocks(n, ORTH_DOT), orth_blocks(n, ORTH_UPD_DOT), orth_blocks(n, ORTH_UPD),
                   orth_blocks(n, ORTH_UPD2), orth_blocks_dot3(n)});
}

int orth_blocks_dot3(int n) { return orth_blocks(n, ORTH_DOT); }

int orth_stride() { return STRIDE; }

hipError_t orth_pass(int mode, const OrthArgs& a, int nblk, hipStream_t s) {
  const int need = a.ncol_max > 0 ? a.ncol_max : a.ncol_fixed + a.ncol_extra;
  if (need > ORTH_MAXCOL) return hipErrorInvalidValue;
  // 16-byte row-pair loads: every column and vector must start 16-byte aligned
  if (a.ld % 2 != 0) return hipErrorInvalidValue;
  const bool nt = static_cast<int64_t>(need) * a.n * 8 >= g_orth_nt_bytes;
  if (a.fuse_norm && (!a.state || !a.norm || (mode != ORTH_UPD && mode != ORTH_UPD2)))
    return hipErrorInvalidValue;
  if (mode == ORTH_UPD) {
    if (nt) hipLaunchKernelGGL(k_upd<true>, dim3(nblk), dim3(UPD_THREADS), 0, s, a);
    else hipLaunchKernelGGL(k_upd<false>, dim3(nblk), dim3(UPD_THREADS), 0, s, a);
    return hipGetLastError();
  }
  if (mode == ORTH_UPD2) {
    if (!a.state || !a.c || !a.Mu || (a.w && (!a.h || !a.wout))) return hipErrorInvalidValue;
    const bool gen = a.Md1 != nullptr && a.Md1 != a.Mu;  // B U corrected too
    if (gen && a.norm) return hipErrorInvalidValue;     // the B-norm needs a product with B
    const dim3 g(nblk), b(UPD_THREADS);
    if (gen) {
      if (nt) hipLaunchKernelGGL((k_upd2<true, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_upd2<false, true>), g, b, 0, s, a);
    } else {
      if (nt) hipLaunchKernelGGL((k_upd2<true, false>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_upd2<false, false>), g, b, 0, s, a);
    }
    return hipGetLastError();
  }
  if (mode == ORTH_DOT && a.nvec == 3) {
    // vec0, vec1 against Md0; vec2 against Md1 (B U for B != I)
    const dim3 g(nblk), b(16 * WAVE);
    const bool same = a.Md1 == nullptr || a.Md1 == a.Md0;
    const bool narrow = (need + 15) / 16 <= 4;
#define TRPLK_DOT3(CPWV, SAMEV)                                                          \
  do {                                                                                   \
    if (nt) hipLaunchKernelGGL((k_orth<CPWV, ORTH_DOT, 3, SAMEV, ORTH_RP, true, 16>), g, b, 0, s, a);  \
    else hipLaunchKernelGGL((k_orth<CPWV, ORTH_DOT, 3, SAMEV, ORTH_RP, false, 16>), g, b, 0, s, a);    \
  } while (0)
    if (narrow && same) TRPLK_DOT3(4, true);
    else if (narrow) TRPLK_DOT3(4, false);
    else if (same) TRPLK_DOT3(8, true);
    else TRPLK_DOT3(8, false);
#undef TRPLK_DOT3
    return hipGetLastError();
  }
  return nt ? launch_width<true>(mode, a, need, nblk, s) : launch_width<false>(mode, a, need, nblk, s);
}

hipError_t finish(const FinishArgs& f, hipStream_t s) {
  if (f.mode == FIN_DC) {
    if (!f.state || !f.T || !f.L || !f.cbuf || (f.nvec == 3 && !f.h)) return hipErrorInvalidValue;
    if (f.cnt < 3 || f.cnt > DC_MAXE || f.stride < f.cnt || f.ldT != SYEV_MAXB) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_finish_dc, dim3(1), dim3(FIN_THREADS), 0, s, f);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(FIN_THREADS), 0, s, f);
  return hipGetLastError();
}

hipError_t set_state(DevState* st, int which, double dv, int iv, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, s, st, which, dv, iv);
  return hipGetLastError();
}

hipError_t set_rho_from(DevState* st, const double* theta, int idx, hipStream_t s) {
  hipLaunchKernelGGL(k_set_rho_from, dim3(1), dim3(1), 0, s, st, theta, idx);
  return hipGetLastError();
}

hipError_t reset_T(double* T, int ldT, int m, int kact, const double* theta, int off, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_T, dim3(16), dim3(256), 0, s, T, ldT, m, kact, theta, off);
  return hipGetLastError();
}

hipError_t ly_product(const double* L, const double* Y, double* YA, int ld, const DevState* st,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_ly, dim3(64), dim3(64), 0, s, L, Y, YA, ld, st);
  return hipGetLastError();
}

hipError_t set_identity(double* L, int ld, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_eye, dim3(16), dim3(256), 0, s, L, ld, m);
  return hipGetLastError();
}

hipError_t restart_residual(int n, const double* AXt, const double* BXt, const double* theta,
                            int t, int next, const double* dinv, double* wout, double* vout,
                            float* vout32, hipStream_t s) {
  hipLaunchKernelGGL(k_restart_residual, dim3(grid1d(n)), dim3(256), 0, s, n, AXt, BXt, theta, t,
                     next, dinv, wout, vout, vout32);
  return hipGetLastError();
}

hipError_t copy_cols(int n, const double* src, int64_t lds, double* dst, int64_t ldd, int ncols,
                     hipStream_t s) {
  if (ncols <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols, dim3(grid1d(static_cast<int64_t>(n) * ncols)), dim3(256), 0, s,
                     n, src, lds, dst, ldd, ncols);
  return hipGetLastError();
}

hipError_t cast_f32(int64_t n, const double* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f32, dim3(grid1d(n)), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

hipError_t cast_f64(int64_t n, const float* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f64, dim3(grid1d(n)), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

hipError_t extract_diag_inv(int n, const int* rowptr, const int* col, const double* val,
                            double* dinv, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_inv, dim3(grid1d(n)), dim3(256), 0, s, n, rowptr, col, val, dinv, bad);
  return hipGetLastError();
}

int rownorm_blocks(int n) { return grid1d(n); }

hipError_t row_norms(int n, const int* rowptr, const double* val, double* partial_inf,
                     double* partial_fro, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_row_norms, dim3(nblk), dim3(256), 0, s, n, rowptr, val, partial_inf,
                     partial_fro);
  return hipGetLastError();
}

}  // namespace trplk
