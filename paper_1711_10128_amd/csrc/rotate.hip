// Thick restart: X = U Y(:, 1:k) for the basis and its products
// (Alg. 1, restart with the k smallest Ritz vectors), in place, with the
// residual norms of the new Ritz pairs computed in the same pass.
//
// This is a dense (n x b) * (b x k) product, so it runs on the FP64 matrix
// cores: each wavefront computes the transposed 16-row output tile
// X(rows,:)^T = Y^T U(rows,:)^T with V_MFMA_F64_16X16X4F64, Y^T fragments in
// registers (or, for the widest bases, read from a copy of Y in LDS) and U
// fragments loaded straight from memory (16 consecutive rows of 4 columns
// per instruction).  The output tile
// layout puts 16 consecutive rows of one column in consecutive lanes, so the
// stores are as contiguous as the loads.  A wavefront reads all b columns of
// its rows before it writes the first k of them, which makes the in-place
// update safe: no other wavefront touches those rows.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace trplk {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int RT = 256;  // threads per block (4 wavefronts)

template <int NTILE, int KS, bool TWOY>
__global__ __launch_bounds__(RT) void k_rotate(const RotArgs a) {
  const int b = a.state ? a.state->nb : a.b_fixed;
  const int kk = min(a.kout, b);
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int li = lane & 15;   // row within the tile / output column of A fragment
  const int lg = lane >> 4;   // k index within a K-step / output row group
  const int64_t ld = a.ld;
  const int n = a.n;
  const bool resid = a.theta && a.AU;

  // A operand (16 outputs x 4 inputs): lane holds Y^T[16 t + li][4 ks + lg].
  // Up to 48 basis columns the fragments stay in registers for the whole
  // kernel; for the widest bases they are read from a copy of Y in LDS just
  // before each product (Y staged once per workgroup, zero outside b x kk),
  // which leaves the register file to the streamed U tiles (measured on
  // MI355X: +33% at b = 64, -5% at b = 40).
  constexpr bool YLDS = KS >= 16;
  __shared__ double Ys[YLDS ? 4 * KS : 1][YLDS ? 16 * NTILE + 1 : 1];
  double yf[NTILE][YLDS ? 1 : KS];
  // TWOY: A U takes its own coefficients YA (delayed re-orthogonalisation
  // keeps uncorrected products; the true ones are AU L), always from LDS
  __shared__ double Ya[TWOY ? 4 * KS : 1][TWOY ? 16 * NTILE + 1 : 1];
  if constexpr (TWOY) {
    for (int e = threadIdx.x; e < 4 * KS * 16 * NTILE; e += RT) {
      const int kin = e % (4 * KS), kout = e / (4 * KS);
      Ya[kin][kout] = (kin < b && kout < kk) ? a.YA[kin + static_cast<int64_t>(kout) * a.ldY] : 0.0;
    }
    if constexpr (!YLDS) __syncthreads();
  }
  if constexpr (YLDS) {
    for (int e = threadIdx.x; e < 4 * KS * 16 * NTILE; e += RT) {
      const int kin = e % (4 * KS), kout = e / (4 * KS);
      Ys[kin][kout] = (kin < b && kout < kk) ? a.Y[kin + static_cast<int64_t>(kout) * a.ldY] : 0.0;
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kin = 4 * ks + lg, kout = 16 * t + li;
        yf[t][ks] = (kin < b && kout < kk) ? a.Y[kin + static_cast<int64_t>(kout) * a.ldY] : 0.0;
      }
    }
  }
  double th[NTILE][4];
  double rs[NTILE][4], xs[NTILE][4];
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kc = 16 * t + lg + 4 * r;
      th[t][r] = (a.theta && kc < kk) ? a.theta[kc] : 0.0;
      rs[t][r] = 0.0;
      xs[t][r] = 0.0;
    }

  // matrices in the order A U, B U, U so that at most two result tiles are
  // live for the residual ||A x - theta B x||
  double* mats[3] = {a.AU, a.BU, a.U};
  const int nwave = gridDim.x * (RT / WAVE);
  const int ntile_rows = (n + 15) / 16;
  for (int rb = blockIdx.x * (RT / WAVE) + wv; rb < ntile_rows; rb += nwave) {
    const int row = rb * 16 + li;
    const bool ok = row < n;
    d4 DA[NTILE];
#pragma unroll
    for (int mi = 0; mi < 3; ++mi) {
      double* M = mats[mi];
      if (M == nullptr) continue;
      // every load unconditional (no branches around them): rows past n and
      // columns past b read a valid entry of the basis instead, whose
      // coefficient in Y is zero, so the products are those of the exact
      // tile; the K steps past b then add exact zeros
      const double* Mrow = M + (ok ? row : n - 1);
      double bv[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kin = min(4 * ks + lg, b - 1);
        bv[ks] = Mrow[kin * ld];
      }
      d4 D[NTILE];
#pragma unroll
      for (int t = 0; t < NTILE; ++t) D[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int t = 0; t < NTILE; ++t)
          D[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              (TWOY && mi == 0) ? Ya[TWOY ? 4 * ks + lg : 0][TWOY ? 16 * t + li : 0]
              : YLDS ? Ys[4 * ks + lg][16 * t + li] : yf[t][YLDS ? 0 : ks],
              bv[ks], D[t], 0, 0, 0);
      }
      // lane holds X(row = rb*16 + li, col = 16 t + lg + 4 r): the F64 16x16x4
      // result places output row lg + 4 r of the tile in register r
#pragma unroll
      for (int t = 0; t < NTILE; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int kc = 16 * t + lg + 4 * r;
          if (ok && kc < kk) M[kc * ld + row] = D[t][r];
        }
      }
      // (rows past n hold products of the stand-in row: kept out of the sums)
      if (resid && ok) {
        if (mi == 0) {
#pragma unroll
          for (int t = 0; t < NTILE; ++t) DA[t] = D[t];
        } else if (mi == 1 || (mi == 2 && a.BU == nullptr)) {
#pragma unroll
          for (int t = 0; t < NTILE; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const double rr = DA[t][r] - th[t][r] * D[t][r];
              rs[t][r] += rr * rr;
            }
        }
        if (mi == 2) {
#pragma unroll
          for (int t = 0; t < NTILE; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) xs[t][r] += D[t][r] * D[t][r];
        }
      }
    }
  }

  if (resid) {
    // sum over the 16 lanes that hold the same output columns
    __shared__ double sr[RT / WAVE][2][64];
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = rs[t][r], w = xs[t][r];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          v += __shfl_xor(v, off, WAVE);
          w += __shfl_xor(w, off, WAVE);
        }
        const int kc = 16 * t + lg + 4 * r;
        if (li == 0 && kc < 64) {
          sr[wv][0][kc] = v;
          sr[wv][1][kc] = w;
        }
      }
    __syncthreads();
    if (threadIdx.x < 64) {
      const int kc = threadIdx.x;
      double v = 0.0, w = 0.0;
      if (kc < 16 * NTILE) {
        for (int q = 0; q < RT / WAVE; ++q) {
          v += sr[q][0][kc];
          w += sr[q][1][kc];
        }
      }
      a.partial[static_cast<int64_t>(blockIdx.x) * 128 + kc] = v;
      a.partial[static_cast<int64_t>(blockIdx.x) * 128 + 64 + kc] = w;
    }
  }
}

template <int NTILE, bool TWOY>
hipError_t launch_nt2(const RotArgs& a, int nblk, hipStream_t s) {
  const int bmax = a.b_max > 0 ? a.b_max : (a.state ? SYEV_MAXB : a.b_fixed);
  const int ks = (bmax + 3) / 4;
  const dim3 g(nblk), b(RT);
  if (ks <= 4) hipLaunchKernelGGL((k_rotate<NTILE, 4, TWOY>), g, b, 0, s, a);
  else if (ks <= 8) hipLaunchKernelGGL((k_rotate<NTILE, 8, TWOY>), g, b, 0, s, a);
  else if (ks <= 12) hipLaunchKernelGGL((k_rotate<NTILE, 12, TWOY>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_rotate<NTILE, 16, TWOY>), g, b, 0, s, a);
  return hipGetLastError();
}

template <int NTILE>
hipError_t launch_nt(const RotArgs& a, int nblk, hipStream_t s) {
  if (a.YA && a.AU) return launch_nt2<NTILE, true>(a, nblk, s);
  return launch_nt2<NTILE, false>(a, nblk, s);
}

}  // namespace

int rot_blocks(int n) {
  const int tiles = (std::max(n, 1) + 15) / 16;
  const int want = (tiles + (RT / WAVE) - 1) / (RT / WAVE);
  return std::max(1, std::min(want, 1024));
}

hipError_t rotate(const RotArgs& a, int nblk, hipStream_t s) {
  switch ((a.kout + 15) / 16) {
    case 1: return launch_nt<1>(a, nblk, s);
    case 2: return launch_nt<2>(a, nblk, s);
    case 3: return launch_nt<3>(a, nblk, s);
    case 4: return launch_nt<4>(a, nblk, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace trplk
