// CSR sparse matrix-vector products (the "MV" of the paper, eq. (3.1)).
//
// The kernels share one epilogue:
//  * CSR-stream (Greathouse and Daga's CSR-Adaptive row blocks, with the
//    block fixed at 64, 32, 16 or 8 rows): when every tile holds at most 512
//    entries, a wavefront loads its tile's contiguous run of values and
//    indices with every lane busy, stages the products in LDS and 64/rows
//    lanes sum each row; this is the kernel for stencil and mesh matrices;
//  * CSR-Adaptive for irregular matrices (power-law graphs): the same tile
//    steps over variable blocks of at most 64 rows and 512 entries listed at
//    plan time; longer rows go to the workgroup-per-row kernel;
//  * row-split (on request of an explicit lane count): a group of L lanes
//    of a wavefront owns one row (L = 2..64,
//    picked from the mean row length), loads its entries coalesced and
//    reduces with cross-lane shuffles; rows of a wavefront are consecutive, so
//    the value and index streams of the wavefront are contiguous;
//  * workgroup-per-row for rows longer than LONG_ROW entries (power-law hubs),
//    listed once at plan time, so a hub row does not stall a wavefront;
//  * diagonal storage for matrices whose entries lie on a few diagonals
//    (stencils and structured meshes): no column indices or row pointers
//    are read, a thread owns a row and reads its value on each diagonal and
//    the shifted x with loads that are contiguous across the wavefront.
// The epilogue fuses the work that touches the row's own entries of the
// dense vectors: scaling by 1/beta, writing the new basis column and its
// products, and forming the next inner direction M (A g - rho B g) for the
// identity and Jacobi preconditioners.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.h"

namespace trplk {

namespace {

constexpr int SPMV_THREADS = 256;
// x staged in LDS for diagonal storage with more than 16 diagonals
bool g_dia_lds = true;
constexpr int DIA_CHUNK = 512;   // rows per block iteration of the staged kernel (two per thread)
constexpr int DIA_LDS_CH = 8;    // diagonal values in flight per thread in the staged kernel

template <typename T>
__device__ __forceinline__ double to_d(T v) {
  return static_cast<double>(v);
}

struct EpiCtx {
  double s;      // scale
  double rho;
  int nb;
};

template <typename OT>
__device__ __forceinline__ void epilogue(const SpmvArgs& a, const EpiCtx& e, int row, double sum,
                                         double& acc) {
  const double yv = e.s * sum;
  switch (a.mode) {
    case SPMV_STORE:
      static_cast<OT*>(a.y)[row] = static_cast<OT>(yv);
      break;
    case SPMV_APPEND: {
      const int64_t c = static_cast<int64_t>(a.col0 + e.nb) * a.ld;
      const double g = e.s * a.xd[row];
      a.U[c + row] = g;
      a.AU[c + row] = yv;
      const double bg = a.bx ? e.s * a.bx[row] : g;
      if (a.BU) a.BU[c + row] = bg;
      if (a.next != NEXT_NONE) {
        const double v = yv - e.rho * bg;
        if (a.next == NEXT_IDENT) {
          a.wout[row] = v;
        } else if (a.next == NEXT_JACOBI) {
          a.wout[row] = a.dinv[row] * v;
        } else {
          if (a.vout32) a.vout32[row] = static_cast<float>(v);
          else a.vout[row] = v;
        }
      }
      break;
    }
    case SPMV_DOT:
      static_cast<OT*>(a.y)[row] = static_cast<OT>(yv);
      acc += yv * a.xd[row];
      break;
    case SPMV_RESID: {
      const double bx = a.bx ? a.bx[row] : a.xd[row];
      const double r = yv - a.theta[a.theta_idx] * bx;
      static_cast<OT*>(a.y)[row] = static_cast<OT>(r);
      acc += r * r;
      break;
    }
  }
}

__device__ __forceinline__ void block_partial(double acc, double* partial, int slot) {
  __shared__ double red[SPMV_THREADS / WAVE];
  acc = wave_sum(acc);
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < SPMV_THREADS / WAVE; ++i) t += red[i];
    partial[slot] = t;
  }
}

// A wavefront owns a tile of 64 consecutive rows.  In sub-iteration q the
// group g of L lanes reduces row q * (64 / L) + g; afterwards the row sums are
// redistributed with shuffles so that lane j holds row j of the tile and the
// epilogue's loads and stores of the dense vectors are fully coalesced.
template <int L, typename VT, typename XT, typename AT, typename OT>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_rows(const SpmvArgs a) {
  EpiCtx e{1.0, 0.0, 0};
  if (a.state) {
    if (a.state->skip) return;
    e.rho = a.state->rho;
    e.nb = a.state->nb;
    if (a.use_beta) e.s = a.state->inv_beta;
  }
  const int* __restrict__ rowptr = a.rowptr;
  const int* __restrict__ col = a.col;
  const VT* __restrict__ val = static_cast<const VT*>(a.val);
  const XT* __restrict__ x = static_cast<const XT*>(a.x);
  constexpr int RPW = WAVE / L;  // rows per sub-iteration
  constexpr int WPB = SPMV_THREADS / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int li = lane & (L - 1);
  const int g = lane / L;
  const int ntile = (a.n + WAVE - 1) / WAVE;
  double acc = 0.0;
  for (int tile = blockIdx.x * WPB + wv; tile < ntile; tile += gridDim.x * WPB) {
    const int r0 = tile * WAVE;
    double mine = 0.0;
    int mylong = 0;
#pragma unroll
    for (int q = 0; q < L; ++q) {
      const int row = r0 + q * RPW + g;
      AT sum = 0;
      int islong = 0;
      if (row < a.n) {
        const int beg = rowptr[row];
        const int end = rowptr[row + 1];
        if (end - beg > LONG_ROW) {
          islong = 1;  // the workgroup-per-row kernel owns it
        } else {
          for (int j = beg + li; j < end; j += L)
            sum += static_cast<AT>(val[j]) * static_cast<AT>(x[col[j]]);
        }
      }
      double sd;
      if constexpr (sizeof(AT) == 4) sd = static_cast<double>(group_sumf<L>(sum));
      else sd = group_sum<L>(sum);
      const int src = (lane % RPW) * L;
      const double t = __shfl(sd, src, WAVE);
      const int tl = __shfl(islong, src, WAVE);
      if (lane / RPW == q) {
        mine = t;
        mylong = tl;
      }
    }
    const int row = r0 + lane;
    if (row < a.n && !mylong) epilogue<OT>(a, e, row, mine, acc);
  }
  if (a.mode == SPMV_DOT || a.mode == SPMV_RESID) block_partial(acc, a.partial, blockIdx.x);
}

// Rows of at most 2L entries (stencils, FEM rows with L = 16): every lane
// handles exactly two entry slots of its row, so the whole 64-row tile's
// loads (row pointers, values, columns, gathers) are straight-line code the
// compiler issues ahead of the arithmetic.
template <int L, typename VT, typename XT, typename AT, typename OT>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_short(const SpmvArgs a) {
  EpiCtx e{1.0, 0.0, 0};
  if (a.state) {
    if (a.state->skip) return;
    e.rho = a.state->rho;
    e.nb = a.state->nb;
    if (a.use_beta) e.s = a.state->inv_beta;
  }
  const int* __restrict__ rowptr = a.rowptr;
  const int* __restrict__ col = a.col;
  const VT* __restrict__ val = static_cast<const VT*>(a.val);
  const XT* __restrict__ x = static_cast<const XT*>(a.x);
  constexpr int RPW = WAVE / L;
  constexpr int WPB = SPMV_THREADS / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int li = lane & (L - 1);
  const int g = lane / L;
  const int ntile = (a.n + WAVE - 1) / WAVE;
  double acc = 0.0;
  for (int tile = blockIdx.x * WPB + wv; tile < ntile; tile += gridDim.x * WPB) {
    const int r0 = tile * WAVE;
    int beg[L], end[L];
#pragma unroll
    for (int q = 0; q < L; ++q) {
      const int row = min(r0 + q * RPW + g, a.n);
      beg[q] = rowptr[row];
      end[q] = row < a.n ? rowptr[row + 1] : beg[q];
    }
    VT v0[L], v1[L];
    int c0[L], c1[L];
#pragma unroll
    for (int q = 0; q < L; ++q) {
      const int j0 = beg[q] + li, j1 = j0 + L;
      const bool k0 = j0 < end[q], k1 = j1 < end[q];
      v0[q] = k0 ? val[j0] : VT(0);
      c0[q] = k0 ? col[j0] : 0;
      v1[q] = k1 ? val[j1] : VT(0);
      c1[q] = k1 ? col[j1] : 0;
    }
    AT s[L];
#pragma unroll
    for (int q = 0; q < L; ++q)
      s[q] = static_cast<AT>(v0[q]) * static_cast<AT>(x[c0[q]]) +
             static_cast<AT>(v1[q]) * static_cast<AT>(x[c1[q]]);
    double mine = 0.0;
#pragma unroll
    for (int q = 0; q < L; ++q) {
      double sd;
      if constexpr (sizeof(AT) == 4) sd = static_cast<double>(group_sumf<L>(s[q]));
      else sd = group_sum<L>(s[q]);
      const double t = __shfl(sd, (lane % RPW) * L, WAVE);
      if (lane / RPW == q) mine = t;
    }
    const int row = r0 + lane;
    if (row < a.n) epilogue<OT>(a, e, row, mine, acc);
  }
  if (a.mode == SPMV_DOT || a.mode == SPMV_RESID) block_partial(acc, a.partial, blockIdx.x);
}

// CSR-stream tile kernel.  A wavefront owns ROWS consecutive rows; the plan
// guarantees that rowptr[r0 + ROWS] - rowptr[r0] <= 64 * KMAX for every
// tile, so the masked loads below cover the whole tile.  Lane i loads
// entries s0+i, s0+i+64, ... and stages the products in LDS; then
// G = 64 / ROWS lanes sum each row's segment (lane rl + ROWS*g takes the
// entries g, g+G, ... of row rl, combined by a fixed shuffle tree) and lane
// rl < ROWS runs the epilogue of row r0 + rl.  The loop is software
// pipelined over the wavefront's tiles: the values and indices of the next
// tile and the row pointers of the one after are loaded while the current
// tile gathers x and sums its rows.
template <int KMAX, int ROWS, typename VT, typename XT, typename AT, typename OT>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_stream(const SpmvArgs a) {
  EpiCtx e{1.0, 0.0, 0};
  if (a.state) {
    if (a.state->skip) return;
    e.rho = a.state->rho;
    e.nb = a.state->nb;
    if (a.use_beta) e.s = a.state->inv_beta;
  }
  constexpr int WPB = SPMV_THREADS / WAVE;
  constexpr int G = WAVE / ROWS;
  __shared__ AT prod[WPB][WAVE * KMAX];
  const int* __restrict__ rowptr = a.rowptr;
  const int* __restrict__ col = a.col;
  const VT* __restrict__ val = static_cast<const VT*>(a.val);
  const XT* __restrict__ x = static_cast<const XT*>(a.x);
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int rl = lane % ROWS;
  const int g = lane / ROWS;
  const int n = a.n;
  const int ntile = (n + ROWS - 1) / ROWS;
  const int stride = gridDim.x * WPB;
  double acc = 0.0;
  // row pointers of tile t (clamped to the last tile past the end)
  auto ptrs = [&](int t, int& rb, int& rt) {
    const int tc = min(t, ntile - 1);
    rb = rowptr[min(tc * ROWS + rl, n)];
    rt = rowptr[min(tc * ROWS + ROWS, n)];
  };
  // values and indices of a tile whose row pointers are rb, rt (none if !live)
  auto entries = [&](bool live, int rb, int rt, VT* v, int* c) {
    const int s0 = __shfl(rb, 0, WAVE);
    const int cnt = live ? rt - s0 : 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const bool ok = lane + WAVE * k < cnt;
      const int idx = s0 + lane + WAVE * k;
      v[k] = ok ? val[idx] : VT(0);
      c[k] = ok ? col[idx] : 0;
    }
  };
  int tile = blockIdx.x * WPB + wv;
  if (tile < ntile) {
    int rb, rt, rbn, rtn;
    VT v[KMAX];
    int c[KMAX];
    ptrs(tile, rb, rt);
    entries(true, rb, rt, v, c);
    int tn = tile + stride;
    ptrs(tn, rbn, rtn);
    while (true) {
      AT pr[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) pr[k] = static_cast<AT>(v[k]) * static_cast<AT>(x[c[k]]);
      const bool more = tn < ntile;
      VT vn[KMAX];
      int cn[KMAX];
      entries(more, rbn, rtn, vn, cn);
      const int t2 = tn + stride;
      int rb2, rt2;
      ptrs(t2, rb2, rt2);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) prod[wv][lane + WAVE * k] = pr[k];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const int s0 = __shfl(rb, 0, WAVE);
      // lanes rl + 1 < ROWS hold the next row's start
      const int nx = __shfl(rb, (rl + 1) & (WAVE - 1), WAVE);
      const int row = tile * ROWS + rl;
      const int end = (rl == ROWS - 1 || row + 1 > n) ? rt : nx;
      AT sum = 0;
      for (int j = rb - s0 + g; j < end - s0; j += G) sum += prod[wv][j];
#pragma unroll
      for (int o = G / 2; o >= 1; o >>= 1) sum += __shfl_xor(sum, o * ROWS, WAVE);
      if (g == 0 && row < n) epilogue<OT>(a, e, row, static_cast<double>(sum), acc);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      if (!more) break;
      tile = tn;
      rb = rbn;
      rt = rtn;
      tn = t2;
      rbn = rb2;
      rtn = rt2;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        v[k] = vn[k];
        c[k] = cn[k];
      }
    }
  }
  if (a.mode == SPMV_DOT || a.mode == SPMV_RESID) block_partial(acc, a.partial, blockIdx.x);
}

// CSR-Adaptive row blocks for irregular matrices: the plan lists blocks of
// at most 64 consecutive rows and 512 entries (rows with more entries go to
// the workgroup-per-row kernel).  The tile steps are those of the stream
// kernel; the number of lanes per row, G, is the largest power of two with
// G * rows <= 64, chosen per block.
template <typename VT, typename XT, typename AT, typename OT>
__device__ __forceinline__ void spmv_adapt_body(const SpmvArgs& a, const int2* blocks, int nblocks,
                                                int bid, int nbid) {
  EpiCtx e{1.0, 0.0, 0};
  if (a.state) {
    if (a.state->skip) return;
    e.rho = a.state->rho;
    e.nb = a.state->nb;
    if (a.use_beta) e.s = a.state->inv_beta;
  }
  constexpr int WPB = SPMV_THREADS / WAVE;
  constexpr int KMAX = ADAPT_MAXNNZ / WAVE;
  __shared__ AT prod[WPB][ADAPT_MAXNNZ];
  const int* __restrict__ rowptr = a.rowptr;
  const int* __restrict__ col = a.col;
  const VT* __restrict__ val = static_cast<const VT*>(a.val);
  const XT* __restrict__ x = static_cast<const XT*>(a.x);
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  double acc = 0.0;
  for (int b = bid * WPB + wv; b < nblocks; b += nbid * WPB) {
    const int2 blk = blocks[b];
    const int r0 = blk.x;
    const int nr = blk.y - blk.x;  // 1..64
    const int rb = rowptr[r0 + min(lane, nr)];
    const int s0 = __shfl(rb, 0, WAVE);
    const int cnt = rowptr[blk.y] - s0;
    VT v[KMAX];
    int c[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const bool ok = lane + WAVE * k < cnt;
      const int idx = s0 + lane + WAVE * k;
      v[k] = ok ? val[idx] : VT(0);
      c[k] = ok ? col[idx] : 0;
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      prod[wv][lane + WAVE * k] = static_cast<AT>(v[k]) * static_cast<AT>(x[c[k]]);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    int G = 1;
    while (2 * G * nr <= WAVE) G *= 2;
    const int rl = lane / G;
    const int g = lane % G;
    // every lane takes part in both shuffles (a lane outside a divergent
    // branch would read as zero); the last row's end is the block's end
    const int lo = __shfl(rb, min(rl, WAVE - 1), WAVE) - s0;
    const int nx = __shfl(rb, min(rl + 1, WAVE - 1), WAVE) - s0;
    const int hi = rl + 1 < nr ? nx : cnt;
    AT sum = 0;
    if (rl < nr)
      for (int j = lo + g; j < hi; j += G) sum += prod[wv][j];
    for (int o = 1; o < G; o <<= 1) sum += __shfl_xor(sum, o, WAVE);
    if (g == 0 && rl < nr) epilogue<OT>(a, e, r0 + rl, static_cast<double>(sum), acc);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
  if (a.mode == SPMV_DOT || a.mode == SPMV_RESID) block_partial(acc, a.partial, bid);
}

template <typename VT, typename XT, typename AT, typename OT>
__device__ __forceinline__ void spmv_long_body(const SpmvArgs& a, const int* long_rows, int slot0,
                                               int bid) {
  EpiCtx e{1.0, 0.0, 0};
  if (a.state) {
    if (a.state->skip) return;
    e.rho = a.state->rho;
    e.nb = a.state->nb;
    if (a.use_beta) e.s = a.state->inv_beta;
  }
  const int row = long_rows[bid];
  const VT* __restrict__ val = static_cast<const VT*>(a.val);
  const XT* __restrict__ x = static_cast<const XT*>(a.x);
  const int beg = a.rowptr[row];
  const int end = a.rowptr[row + 1];
  AT sum = 0;
  for (int j = beg + threadIdx.x; j < end; j += SPMV_THREADS)
    sum += static_cast<AT>(val[j]) * static_cast<AT>(x[a.col[j]]);
  __shared__ double red[SPMV_THREADS / WAVE];
  double s = wave_sum(static_cast<double>(sum));
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < SPMV_THREADS / WAVE; ++i) t += red[i];
    double acc = 0.0;
    epilogue<OT>(a, e, row, t, acc);
    if (a.mode == SPMV_DOT || a.mode == SPMV_RESID) a.partial[slot0 + bid] = acc;
  }
}

template <typename VT, typename XT, typename AT, typename OT>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_long(const SpmvArgs a, const int* long_rows,
                                                            int slot0) {
  spmv_long_body<VT, XT, AT, OT>(a, long_rows, slot0, blockIdx.x);
}

// CSR-Adaptive blocks and the long rows in one launch: the first nlong
// workgroups take one long row each (they start first, so a hub row does
// not trail the launch), the rest step over the adaptive blocks.  Partial
// slots: adaptive workgroup j -> j, long row i -> nadapt + i.
template <typename VT, typename XT, typename AT, typename OT>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_adapt_long(const SpmvArgs a,
                                                                  const int2* blocks, int nblocks,
                                                                  int nadapt, const int* long_rows,
                                                                  int nlong) {
  const int bid = blockIdx.x;
  if (bid < nlong) spmv_long_body<VT, XT, AT, OT>(a, long_rows, nadapt, bid);
  else spmv_adapt_body<VT, XT, AT, OT>(a, blocks, nblocks, bid - nlong, nadapt);
}

// Row lengths: long-row flags, the longest row and the fullest tile of
// 64, 32, 16 and 8 rows (maxtile[0..3]).
__global__ void k_find_long(int n, const int* rowptr, int* flags, int* maxlen, int* maxtile) {
  int mx = 0, mt[4] = {0, 0, 0, 0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int len = rowptr[i + 1] - rowptr[i];
    flags[i] = len > LONG_ROW;
    mx = max(mx, len);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rows = WAVE >> q;
      if (i % rows == 0) mt[q] = max(mt[q], rowptr[min(i + rows, n)] - rowptr[i]);
    }
  }
  atomicMax(maxlen, mx);
#pragma unroll
  for (int q = 0; q < 4; ++q) atomicMax(maxtile + q, mt[q]);
}

// Diagonal storage: thread i of the grid-stride loop owns row i; the row
// sum runs over the diagonals in ascending offset order (ascending column),
// skipping the zeros that pad the diagonals; x is read at the clamped
// column, which only the padding ever needs.  MAXD bounds the unrolled
// diagonal count (ndiag <= MAXD).
// Chunks of 256 rows for the diagonal kernels.  XCD: workgroups are
// dispatched to the eight XCDs in turn (workgroup b on XCD b mod 8), each
// with its own L2; with a grid that is a multiple of 8 every XCD takes a
// contiguous eighth of the chunks, its workgroups striding through it
// together, so the rows a chunk shares with its neighbours stay in one L2.
// Used with LDS staging (27-point stencils: 3% on the 97^3 FEM pencil
// together with the non-temporal value loads); the unstaged kernel keeps the
// plain grid stride (no gain measured on the 7-point operators).
struct ChunkRange {
  int first, end, step;
};

template <bool XCD>
__device__ __forceinline__ ChunkRange dia_chunks(int nchunk) {
  if (XCD && (gridDim.x & 7) == 0) {
    const int per = static_cast<int>(gridDim.x) >> 3;
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int cx = (nchunk + 7) / 8;
    return {xcd * cx + local, min(nchunk, (xcd + 1) * cx), per};
  }
  return {static_cast<int>(blockIdx.x), nchunk, static_cast<int>(gridDim.x)};
}

// NT: non-temporal loads of the diagonal values, which are read once.
// Measured on MI355X: the staged 27-diagonal product gains 4%, but on the
// 7-point 256^3 operator the unstaged product's 5% gain came with a 3%
// slower solve (the kernels around it lost more), so only the staged kernel
// uses them.
template <bool NT, typename VT>
__device__ __forceinline__ VT ld_val(const VT* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <int MAXD, typename VT, typename XT, typename AT, typename OT>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_dia(const SpmvArgs a, const int* __restrict__ off,
                                                        int ndiag, const VT* __restrict__ dval) {
  EpiCtx e{1.0, 0.0, 0};
  if (a.state) {
    if (a.state->skip) return;
    e.rho = a.state->rho;
    e.nb = a.state->nb;
    if (a.use_beta) e.s = a.state->inv_beta;
  }
  const XT* __restrict__ x = static_cast<const XT*>(a.x);
  const int n = a.n;
  int o[MAXD];
#pragma unroll
  for (int d = 0; d < MAXD; ++d) o[d] = d < ndiag ? off[d] : 0;
  double acc = 0.0;
  if constexpr (MAXD <= 8 && sizeof(VT) == 8) {
    // float64 values: two rows per thread, SPMV_THREADS apart (chunks of
    // 2 * SPMV_THREADS rows), so twice the loads are in flight per wavefront;
    // each row's sum and epilogue are those of the one-row form.  Measured
    // on the 256^3 operator: A products 117 -> 113 ms and float64 FSAI
    // applies 111 -> 101 ms per 10 cycles; with float32 values the same form
    // is slower (factor applies 60 -> 77 ms), so those keep one row.
    const ChunkRange c2 = dia_chunks<false>((n + 2 * SPMV_THREADS - 1) / (2 * SPMV_THREADS));
    for (int ch = c2.first; ch < c2.end; ch += c2.step) {
      const int r0 = ch * 2 * SPMV_THREADS + threadIdx.x;
      if (r0 >= n) continue;
      const int r1 = r0 + SPMV_THREADS;
      const bool ok1 = r1 < n;
      const int r1c = ok1 ? r1 : r0;  // past the end: row r0 again, not used
      VT v0[MAXD], v1[MAXD];
      XT x0[MAXD], x1[MAXD];
#pragma unroll
      for (int d = 0; d < MAXD; ++d) {
        if (d < ndiag) {
          v0[d] = ld_val<false>(dval + static_cast<int64_t>(d) * n + r0);
          v1[d] = ld_val<false>(dval + static_cast<int64_t>(d) * n + r1c);
          const int64_t c0 = static_cast<int64_t>(r0) + o[d];
          const int64_t c1 = static_cast<int64_t>(r1c) + o[d];
          x0[d] = x[c0 < 0 ? 0 : (c0 >= n ? n - 1 : c0)];
          x1[d] = x[c1 < 0 ? 0 : (c1 >= n ? n - 1 : c1)];
        }
      }
      // zero entries add 0 * x[clamped] = 0, as below
      AT s0 = 0, s1 = 0;
#pragma unroll
      for (int d = 0; d < MAXD; ++d)
        if (d < ndiag) {
          s0 += static_cast<AT>(v0[d]) * static_cast<AT>(x0[d]);
          s1 += static_cast<AT>(v1[d]) * static_cast<AT>(x1[d]);
        }
      epilogue<OT>(a, e, r0, static_cast<double>(s0), acc);
      if (ok1) epilogue<OT>(a, e, r1, static_cast<double>(s1), acc);
    }
    if (a.mode == SPMV_DOT || a.mode == SPMV_RESID) block_partial(acc, a.partial, blockIdx.x);
    return;
  }
  const ChunkRange cr = dia_chunks<false>((n + SPMV_THREADS - 1) / SPMV_THREADS);
  for (int ch = cr.first; ch < cr.end; ch += cr.step) {
    const int row = ch * SPMV_THREADS + threadIdx.x;
    if (row >= n) continue;
    AT sum = 0;
    if constexpr (MAXD <= 8) {
      VT v[MAXD];
      XT xv[MAXD];
#pragma unroll
      for (int d = 0; d < MAXD; ++d) {
        if (d < ndiag) {
          v[d] = ld_val<false>(dval + static_cast<int64_t>(d) * n + row);
          const int64_t c = static_cast<int64_t>(row) + o[d];
          xv[d] = x[c < 0 ? 0 : (c >= n ? n - 1 : c)];
        }
      }
      // zero entries (the padding of diagonals that leave the matrix) add
      // 0 * x[clamped] = 0: no per-lane branch, the same sums
#pragma unroll
      for (int d = 0; d < MAXD; ++d)
        if (d < ndiag) sum += static_cast<AT>(v[d]) * static_cast<AT>(xv[d]);
    } else {
      // diagonals in chunks of 8, the loads of a chunk in flight together:
      // fewer registers than holding every diagonal's loads keep more
      // wavefronts resident (the same summation order)
#pragma unroll 1
      for (int d0 = 0; d0 < MAXD; d0 += 8) {
        if (d0 >= ndiag) break;
        VT v[8];
        XT xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int d = d0 + q;
          if (d < ndiag) {
            v[q] = ld_val<false>(dval + static_cast<int64_t>(d) * n + row);
            const int64_t c = static_cast<int64_t>(row) + o[d];
            xv[q] = x[c < 0 ? 0 : (c >= n ? n - 1 : c)];
          }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (d0 + q < ndiag) sum += static_cast<AT>(v[q]) * static_cast<AT>(xv[q]);  // zeros add 0
      }
    }
    epilogue<OT>(a, e, row, static_cast<double>(sum), acc);
  }
  if (a.mode == SPMV_DOT || a.mode == SPMV_RESID) block_partial(acc, a.partial, blockIdx.x);
}

// The same product with x staged in LDS.  A block owns DIA_CHUNK = 512
// consecutive rows per iteration, two adjacent rows per thread (one 16-byte
// load of each diagonal's pair of values when n is even; 256 rows, one per
// thread: 1.6% slower; 1024 rows, four per thread 256 apart: 11% slower),
// the chunks taken XCD by XCD; the column offsets fall into a few clusters
// (a stencil's planes: the 27-point operator has three, each 195 rows
// wide), and the block loads each cluster's window of x (512 + span
// entries, coalesced) once, so the ndiag shifted reads of a row come from
// LDS instead of the cache hierarchy.  Values, the summation order of each
// row and the epilogue are those of k_spmv_dia, so the products are
// identical (the fused dot of SPMV_DOT / SPMV_RESID groups the rows per
// thread and block differently).  Used for more than 16 diagonals: with
// fewer (the FSAI factors' 14) the staging costs more than the reads it
// saves (measured); 8 values in flight per row (16: the same, 32: 5%
// slower).
struct DiaStage {
  int ncl;
  int lo[8];
  int len[8];
  int base[8];
  int doff[32];
};

template <int MAXD, typename VT, typename XT, typename AT, typename OT>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_dia_lds(const SpmvArgs a, int ndiag,
                                                            const VT* __restrict__ dval,
                                                            const DiaStage ds) {
  extern __shared__ char lds_raw[];
  XT* xs = reinterpret_cast<XT*>(lds_raw);
  EpiCtx e{1.0, 0.0, 0};
  if (a.state) {
    if (a.state->skip) return;
    e.rho = a.state->rho;
    e.nb = a.state->nb;
    if (a.use_beta) e.s = a.state->inv_beta;
  }
  const XT* __restrict__ x = static_cast<const XT*>(a.x);
  const int n = a.n;
  double acc = 0.0;
  const ChunkRange cr = dia_chunks<true>((n + DIA_CHUNK - 1) / DIA_CHUNK);
  for (int ch = cr.first; ch < cr.end; ch += cr.step) {
    const int r0 = ch * DIA_CHUNK;
    for (int c = 0; c < ds.ncl; ++c) {
      const int64_t g0 = static_cast<int64_t>(r0) + ds.lo[c];
      for (int t = threadIdx.x; t < ds.len[c]; t += SPMV_THREADS) {
        const int64_t gi = g0 + t;
        xs[ds.base[c] + t] = (gi >= 0 && gi < n) ? x[gi] : XT(0);
      }
    }
    __syncthreads();
    {
      typedef VT VT2 __attribute__((ext_vector_type(2)));
      const int loc = 2 * threadIdx.x;
      const int row = r0 + loc;
      if (row < n) {
        const bool two = row + 1 < n;
        const bool vec = two && (n & 1) == 0;
        AT s0 = 0, s1 = 0;
#pragma unroll 1
        for (int d0 = 0; d0 < MAXD; d0 += DIA_LDS_CH) {
          if (d0 >= ndiag) break;
          VT v0[DIA_LDS_CH], v1[DIA_LDS_CH];
#pragma unroll
          for (int q = 0; q < DIA_LDS_CH; ++q)
            if (d0 + q < ndiag) {
              const VT* p = dval + static_cast<int64_t>(d0 + q) * n + row;
              if (vec) {
                const VT2 pr = __builtin_nontemporal_load(reinterpret_cast<const VT2*>(p));
                v0[q] = pr.x;
                v1[q] = pr.y;
              } else {
                v0[q] = ld_val<true>(p);
                v1[q] = two ? ld_val<true>(p + 1) : VT(0);
              }
            }
#pragma unroll
          for (int q = 0; q < DIA_LDS_CH; ++q) {
            const int d = d0 + q;
            if (d < ndiag) {
              // zero entries add 0 (the staged x is finite, 0 outside the vector)
              s0 += static_cast<AT>(v0[q]) * static_cast<AT>(xs[ds.doff[d] + loc]);
              s1 += static_cast<AT>(v1[q]) * static_cast<AT>(xs[ds.doff[d] + loc + 1]);
            }
          }
        }
        epilogue<OT>(a, e, row, static_cast<double>(s0), acc);
        if (two) epilogue<OT>(a, e, row + 1, static_cast<double>(s1), acc);
      }
    }
    __syncthreads();
  }
  if (a.mode == SPMV_DOT || a.mode == SPMV_RESID) block_partial(acc, a.partial, blockIdx.x);
}

// scatter of the CSR values into diagonal storage (zeroed beforehand): one
// thread per row; repeated entries of a position are summed, as the CSR
// kernels do
template <typename VT>
__global__ void k_dia_fill(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                           const VT* __restrict__ val, const int* __restrict__ off, int ndiag,
                           VT* __restrict__ dval) {
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < n; row += gridDim.x * blockDim.x) {
    for (int k = rowptr[row]; k < rowptr[row + 1]; ++k) {
      const int o = col[k] - row;
      int d = 0;
      while (d < ndiag - 1 && off[d] != o) ++d;  // every offset is listed (checked on the host)
      dval[static_cast<int64_t>(d) * n + row] += val[k];
    }
  }
}

template <typename VT, typename XT, typename AT, typename OT>
hipError_t launch_dia(const SpmvPlan& p, const SpmvArgs& a, const VT* dval, hipStream_t s) {
  if (!dval) return hipErrorInvalidValue;  // this precision was not prepared
  const dim3 grd(p.nblk_dia), blk(SPMV_THREADS);
  if (p.ncl > 0 && g_dia_lds && p.ndiag > 16) {
    DiaStage ds{};
    ds.ncl = p.ncl;
    for (int c = 0; c < p.ncl; ++c) {
      ds.lo[c] = p.cl_lo[c];
      ds.len[c] = p.cl_len[c];
      ds.base[c] = p.cl_base[c];
    }
    for (int d = 0; d < p.ndiag; ++d) ds.doff[d] = p.doff[d];
    const size_t shm = sizeof(XT) * static_cast<size_t>(p.lds_elems);
    // the grid of the unstaged kernel: every partial slot the reductions read
    // is written (blocks past the last chunk write zero)
    hipLaunchKernelGGL((k_spmv_dia_lds<DIA_MAXD, VT, XT, AT, OT>), grd, blk, shm, s, a, p.ndiag, dval, ds);
    return hipGetLastError();
  }
  if (p.ndiag <= 8)
    hipLaunchKernelGGL((k_spmv_dia<8, VT, XT, AT, OT>), grd, blk, 0, s, a, p.dia_off, p.ndiag, dval);
  else if (p.ndiag <= 16)
    hipLaunchKernelGGL((k_spmv_dia<16, VT, XT, AT, OT>), grd, blk, 0, s, a, p.dia_off, p.ndiag, dval);
  else
    hipLaunchKernelGGL((k_spmv_dia<DIA_MAXD, VT, XT, AT, OT>), grd, blk, 0, s, a, p.dia_off, p.ndiag,
                       dval);
  return hipGetLastError();
}

void dia_free(SpmvPlan& plan) {
  if (plan.dia_off) (void)hipFree(plan.dia_off);
  if (plan.dia_val) (void)hipFree(plan.dia_val);
  if (plan.dia_val32) (void)hipFree(plan.dia_val32);
  plan.dia_off = nullptr;
  plan.dia_val = nullptr;
  plan.dia_val32 = nullptr;
  plan.ndiag = 0;
  plan.nblk_dia = 0;
  plan.ncl = 0;
  plan.lds_elems = 0;
}

// Grid of the tile kernels: one tile per wavefront up to a cap.  The
// software-pipelined CSR-stream kernel runs best with two rounds of resident
// blocks (16 blocks of 4 wavefronts per compute unit, measured on MI355X for
// the 27-point and 7-point matrices); the row-split kernels with a deeper grid.
int short_blocks(int n, bool stream, int rows = WAVE) {
  const int tiles = (n + rows - 1) / rows;
  const int want = (tiles + SPMV_THREADS / WAVE - 1) / (SPMV_THREADS / WAVE);
  return std::max(1, std::min(want, stream ? 4096 : 8192));
}

template <typename VT, typename XT, typename AT, typename OT>
hipError_t launch(const SpmvPlan& p, const SpmvArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (p.ndiag > 0) {
    if constexpr (std::is_same<VT, double>::value) return launch_dia<VT, XT, AT, OT>(p, a, p.dia_val, s);
    else return launch_dia<VT, XT, AT, OT>(p, a, p.dia_val32, s);
  }
  const dim3 blk(SPMV_THREADS);
  const dim3 grd(p.nblk_short);
  if (p.nblocks > 0 || p.adaptive) {
    // with no adaptive blocks the adaptive workgroups find no work; their
    // partial slots are still written (zero) for the dot epilogues
    hipLaunchKernelGGL((k_spmv_adapt_long<VT, XT, AT, OT>), dim3(p.nlong + p.nblk_short), blk, 0, s,
                       a, p.blocks, p.nblocks, p.nblk_short, p.long_rows, p.nlong);
    return hipGetLastError();
  }
  if (p.kmax == 8) {
    switch (p.tile_rows) {
      case 64: hipLaunchKernelGGL((k_spmv_stream<8, 64, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
      case 32: hipLaunchKernelGGL((k_spmv_stream<8, 32, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
      case 16: hipLaunchKernelGGL((k_spmv_stream<8, 16, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
      default: hipLaunchKernelGGL((k_spmv_stream<8, 8, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
    }
    return hipGetLastError();
  }
  // two entry slots per lane cover every row: the straight-line kernel with
  // exactly p.lanes lanes per row (2..32; wider rows use the loop kernel)
  if (p.nlong == 0 && p.maxlen <= 2 * p.lanes && p.lanes >= 2 && p.lanes <= 32) {
    switch (p.lanes) {
      case 2: hipLaunchKernelGGL((k_spmv_short<2, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((k_spmv_short<4, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
      case 8: hipLaunchKernelGGL((k_spmv_short<8, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
      case 16: hipLaunchKernelGGL((k_spmv_short<16, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
      case 32: hipLaunchKernelGGL((k_spmv_short<32, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;  // lane counts are powers of two
    }
    return hipGetLastError();
  }
  switch (p.lanes) {
    case 1: hipLaunchKernelGGL((k_spmv_rows<1, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_spmv_rows<2, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_spmv_rows<4, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_spmv_rows<8, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_spmv_rows<16, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_spmv_rows<32, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
    default: hipLaunchKernelGGL((k_spmv_rows<64, VT, XT, AT, OT>), grd, blk, 0, s, a); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.nlong > 0) {
    hipLaunchKernelGGL((k_spmv_long<VT, XT, AT, OT>), dim3(p.nlong), blk, 0, s, a, p.long_rows,
                       p.nblk_short);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace

// Lanes per row: the smallest power of two covering half the mean row
// length (two loads per lane for a typical row; measured best for the
// 7-point stencil: 4 lanes).
int pick_lanes(double mean_len) {
  int L = 2;
  while (L < 64 && 2 * L < mean_len) L <<= 1;
  return L;
}

// Irregular matrices: blocks of consecutive rows with at most 64 rows and
// ADAPT_MAXNNZ entries, built on the host from a copy of the row pointers;
// rows longer than ADAPT_MAXNNZ entries are listed for the long-row kernel.
hipError_t adaptive_plan(SpmvPlan& plan, int n, const int* rowptr_dev, hipStream_t s) {
  std::vector<int> rp(static_cast<size_t>(n) + 1);
  hipError_t e = hipMemcpyAsync(rp.data(), rowptr_dev, sizeof(int) * (n + 1),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  std::vector<int2> blocks;
  std::vector<int> longs;
  int i = 0;
  while (i < n) {
    if (rp[i + 1] - rp[i] > ADAPT_MAXNNZ) {
      longs.push_back(i++);
      continue;
    }
    int j = i + 1;
    while (j < n && j - i < WAVE && rp[j + 1] - rp[i] <= ADAPT_MAXNNZ) ++j;
    blocks.push_back(make_int2(i, j));
    i = j;
  }
  plan.adaptive = true;
  plan.nblocks = static_cast<int>(blocks.size());
  plan.nlong = static_cast<int>(longs.size());
  plan.nblk_short = std::max(1, std::min((plan.nblocks + 3) / 4, 2048));
  if (plan.nblocks) {
    e = hipMalloc(&plan.blocks, sizeof(int2) * blocks.size());
    if (e == hipSuccess)
      e = hipMemcpyAsync(plan.blocks, blocks.data(), sizeof(int2) * blocks.size(),
                         hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess && plan.nlong) {
    e = hipMalloc(&plan.long_rows, sizeof(int) * longs.size());
    if (e == hipSuccess)
      e = hipMemcpyAsync(plan.long_rows, longs.data(), sizeof(int) * longs.size(),
                         hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

hipError_t spmv_plan(SpmvPlan& plan, int n, const int* rowptr_dev, int lanes, hipStream_t s) {
  dia_free(plan);
  plan.n = n;
  int nnz = 0;
  hipError_t e = hipSuccess;
  if (n > 0) {
    e = hipMemcpyAsync(&nnz, rowptr_dev + n, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
  }
  plan.lanes = lanes > 0 ? lanes : pick_lanes(n ? double(nnz) / n : 1.0);
  plan.kmax = 0;
  plan.tile_rows = WAVE;
  plan.adaptive = false;
  plan.nblocks = 0;
  plan.blocks = nullptr;
  plan.nblk_short = short_blocks(std::max(n, 1), false);
  plan.nlong = 0;
  plan.long_rows = nullptr;
  if (n == 0) return hipSuccess;
  int* flags = nullptr;
  e = hipMalloc(&flags, sizeof(int) * (n + 5));
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(flags + n, 0, 5 * sizeof(int), s);
  if (e != hipSuccess) {
    (void)hipFree(flags);
    return e;
  }
  hipLaunchKernelGGL(k_find_long, dim3(std::min((n + 255) / 256, 4096)), dim3(256), 0, s, n,
                     rowptr_dev, flags, flags + n, flags + n + 1);
  std::vector<int> h(n + 5);
  e = hipMemcpyAsync(h.data(), flags, sizeof(int) * (n + 5), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(flags);
  plan.maxlen = h[n];
  plan.maxtile = h[n + 1];
  if (e != hipSuccess) return e;
  // CSR-stream with the tallest tile (64, 32, 16 or 8 rows) that never
  // exceeds 512 entries; an explicit lane count asks for the row-split kernels
  if (lanes <= 0) {
    for (int q = 0; q < 4; ++q) {
      if (h[n + 1 + q] <= WAVE * 8) {
        plan.kmax = 8;
        plan.tile_rows = WAVE >> q;
        break;
      }
    }
    if (plan.kmax) {
      plan.nblk_short = short_blocks(n, true, plan.tile_rows);
      return hipSuccess;  // the stream kernel covers long rows too
    }
    return adaptive_plan(plan, n, rowptr_dev, s);
  }
  std::vector<int> rows;
  for (int i = 0; i < n; ++i)
    if (h[i]) rows.push_back(i);
  plan.nlong = static_cast<int>(rows.size());
  if (plan.nlong) {
    e = hipMalloc(&plan.long_rows, sizeof(int) * rows.size());
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(plan.long_rows, rows.data(), sizeof(int) * rows.size(),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  return e;
}

hipError_t spmv_plan_dia(SpmvPlan& plan, int n, const int* rowptr_dev, const int* col_dev,
                         const double* val64, const float* val32, hipStream_t s) {
  dia_free(plan);
  if (n <= 0 || (!val64 && !val32)) return hipSuccess;
  std::vector<int> rp(static_cast<size_t>(n) + 1);
  hipError_t e = hipMemcpyAsync(rp.data(), rowptr_dev, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const int64_t nnz = rp[n];
  if (rp[0] != 0 || nnz <= 0) return hipSuccess;  // keep CSR
  // the diagonal format reads 8 bytes per diagonal and row against CSR's 12
  // per entry plus 4 per row: used only at or below 85% of the CSR bytes
  const int64_t max_d =
      std::min<int64_t>(DIA_MAXD, (85 * (12 * nnz + 4 * (int64_t(n) + 1))) / (100 * 8 * int64_t(n)));
  if (max_d < 1) return hipSuccess;
  std::vector<int> cl(static_cast<size_t>(nnz));
  e = hipMemcpyAsync(cl.data(), col_dev, sizeof(int) * nnz, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  std::vector<int> offs;
  for (int i = 0; i < n; ++i) {
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int o = cl[k] - i;
      if (std::find(offs.begin(), offs.end(), o) == offs.end()) {
        offs.push_back(o);
        if (static_cast<int64_t>(offs.size()) > max_d) return hipSuccess;  // CSR stays
      }
    }
  }
  std::sort(offs.begin(), offs.end());
  const int nd = static_cast<int>(offs.size());
  const int64_t cells = static_cast<int64_t>(nd) * n;
  e = hipMalloc(&plan.dia_off, sizeof(int) * nd);
  if (e == hipSuccess) e = hipMemcpyAsync(plan.dia_off, offs.data(), sizeof(int) * nd, hipMemcpyHostToDevice, s);
  const int grid = std::min((n + 255) / 256, 4096);
  if (e == hipSuccess && val64) {
    e = hipMalloc(&plan.dia_val, sizeof(double) * cells);
    if (e == hipSuccess) e = hipMemsetAsync(plan.dia_val, 0, sizeof(double) * cells, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_dia_fill<double>, dim3(grid), dim3(256), 0, s, n, rowptr_dev, col_dev, val64,
                         plan.dia_off, nd, plan.dia_val);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess && val32) {
    e = hipMalloc(&plan.dia_val32, sizeof(float) * cells);
    if (e == hipSuccess) e = hipMemsetAsync(plan.dia_val32, 0, sizeof(float) * cells, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_dia_fill<float>, dim3(grid), dim3(256), 0, s, n, rowptr_dev, col_dev, val32,
                         plan.dia_off, nd, plan.dia_val32);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dia_free(plan);
    return e;
  }
  plan.ndiag = nd;
  // every block resident at once: 8 blocks of 4 wavefronts per compute unit
  plan.nblk_dia = std::max(1, std::min((n + SPMV_THREADS - 1) / SPMV_THREADS, 2048));
  // LDS staging of x: split the sorted offsets where consecutive ones are
  // more than a chunk apart; each cluster's window is the chunk plus its span
  {
    int ncl = 0, total = 0;
    bool ok = true;
    int c0 = 0;
    for (int d = 0; d <= nd && ok; ++d) {
      if (d == nd || (d > c0 && offs[d] - offs[d - 1] > SPMV_THREADS)) {
        if (ncl == 8) { ok = false; break; }
        plan.cl_lo[ncl] = offs[c0];
        plan.cl_len[ncl] = DIA_CHUNK + offs[d - 1] - offs[c0];
        plan.cl_base[ncl] = total;
        for (int q = c0; q < d; ++q) plan.doff[q] = total + offs[q] - offs[c0];
        total += plan.cl_len[ncl];
        ++ncl;
        c0 = d;
      }
    }
    // at most 4096 entries of windows per block (32 KiB of LDS in float64)
    if (ok && total <= 4096) {
      plan.ncl = ncl;
      plan.lds_elems = total;
    } else {
      plan.ncl = 0;
    }
  }
  return hipSuccess;
}

int64_t spmv_matrix_bytes(const SpmvPlan& plan, int64_t nnz, bool f32) {
  const int64_t vb = f32 ? 4 : 8;
  if (plan.ndiag > 0) return vb * plan.ndiag * static_cast<int64_t>(plan.n);
  return nnz * (vb + 4) + 4 * (static_cast<int64_t>(plan.n) + 1);
}

void spmv_plan_free(SpmvPlan& plan) {
  if (plan.long_rows) (void)hipFree(plan.long_rows);
  if (plan.blocks) (void)hipFree(plan.blocks);
  plan.long_rows = nullptr;
  plan.blocks = nullptr;
  plan.nlong = 0;
  plan.nblocks = 0;
  dia_free(plan);
}

int spmv_partial_blocks(const SpmvPlan& plan) {
  if (plan.ndiag > 0) return plan.nblk_dia;
  return plan.kmax ? plan.nblk_short : plan.nblk_short + plan.nlong;
}

namespace {

// Y(:, j) = A X(:, j) for the s <= S columns a block of block TRPL+K has
// appended, A in diagonal storage (float64): each diagonal value is read
// once for all columns.  A row's sum over the diagonals runs in ascending
// order; zero entries are skipped here and add exact zeros in k_spmv_dia
// (x finite), so every column equals that kernel's product bit for bit.
template <int S>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmm_dia(int n, int ndiag, const int* __restrict__ off,
                                                        const double* __restrict__ dval,
                                                        const double* __restrict__ X, int64_t ldx, int s,
                                                        double* __restrict__ Y, int64_t ldy) {
  __shared__ int so[DIA_MAXD];
  for (int d = threadIdx.x; d < ndiag; d += SPMV_THREADS) so[d] = off[d];
  __syncthreads();
  for (int row = blockIdx.x * SPMV_THREADS + threadIdx.x; row < n; row += gridDim.x * SPMV_THREADS) {
    double acc[S];
#pragma unroll
    for (int j = 0; j < S; ++j) acc[j] = 0.0;
    for (int d = 0; d < ndiag; ++d) {
      const double v = dval[static_cast<int64_t>(d) * n + row];
      if (v != 0.0) {
        const int64_t c = static_cast<int64_t>(row) + so[d];   // in range where v != 0
#pragma unroll
        for (int j = 0; j < S; ++j)
          if (j < s) acc[j] += v * X[static_cast<int64_t>(j) * ldx + c];
      }
    }
#pragma unroll
    for (int j = 0; j < S; ++j)
      if (j < s) Y[static_cast<int64_t>(j) * ldy + row] = acc[j];
  }
}

}  // namespace

bool spmm_dia_ready(const SpmvPlan& plan) { return plan.ndiag > 0 && plan.dia_val != nullptr; }

hipError_t spmm_dia(const SpmvPlan& plan, int n, const double* X, int64_t ldx, int ncols, double* Y,
                    int64_t ldy, hipStream_t s) {
  if (!spmm_dia_ready(plan) || ncols < 1 || ncols > 16 || n < 1) return hipErrorInvalidValue;
  const dim3 g(plan.nblk_dia), b(SPMV_THREADS);
  if (ncols <= 2)
    hipLaunchKernelGGL(k_spmm_dia<2>, g, b, 0, s, n, plan.ndiag, plan.dia_off, plan.dia_val, X, ldx, ncols, Y, ldy);
  else if (ncols <= 4)
    hipLaunchKernelGGL(k_spmm_dia<4>, g, b, 0, s, n, plan.ndiag, plan.dia_off, plan.dia_val, X, ldx, ncols, Y, ldy);
  else if (ncols <= 8)
    hipLaunchKernelGGL(k_spmm_dia<8>, g, b, 0, s, n, plan.ndiag, plan.dia_off, plan.dia_val, X, ldx, ncols, Y, ldy);
  else
    hipLaunchKernelGGL(k_spmm_dia<16>, g, b, 0, s, n, plan.ndiag, plan.dia_off, plan.dia_val, X, ldx, ncols, Y,
                       ldy);
  return hipGetLastError();
}

hipError_t spmv_f64(const SpmvPlan& plan, const SpmvArgs& a, hipStream_t s) {
  return launch<double, double, double, double>(plan, a, s);
}

// float32 values and gather vector with float32 accumulation; the epilogue
// writes float32 (or float64 when out_f64) for SPMV_STORE / SPMV_DOT and
// float64 columns for SPMV_APPEND.
hipError_t spmv_f32(const SpmvPlan& plan, const SpmvArgs& a, hipStream_t s) {
  if (a.out_f64) return launch<float, float, float, double>(plan, a, s);
  return launch<float, float, float, float>(plan, a, s);
}

}  // namespace trplk
