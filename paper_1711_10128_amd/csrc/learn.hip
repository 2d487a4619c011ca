// Learned factorized preconditioner M = G^T G: row features, the two-layer
// MLP that predicts G on the lower pattern of A, and its training kernels.
//
// Network (per lower-triangular nonzero (i, j) of A, float32):
//   x = [f_i (8), f_j (8), |a_ij| / sqrt(a_ii a_jj)]          (17 inputs)
//   h = relu(W1 x + b1)  (64),   o = w2 . h + b2
//   G(i,i) = exp(o) / sqrt(a_ii),   G(i,j) = -o a_ij / (cbar a_jj sqrt(a_ii))  (j < i)
// with cbar the mean normalised coupling |a_ij| / sqrt(a_ii a_jj) over the
// strictly lower entries, so G has a positive diagonal (M is SPD by
// construction) and a zero output layer gives G = D^{-1/2}, i.e. the Jacobi
// preconditioner.  Up to the constant cbar the off-diagonal scale is that of
// a first-order factor (o = cbar off the diagonal, 0 on it, gives
// D^{-1/2}(I - L D^{-1}), L the strict lower triangle, the expansion of the
// symmetric Gauss-Seidel factor D^{1/2}(D + L)^{-1}): a column j shared by
// many rows (a graph hub) enters G^T with weights falling as 1/a_jj, so the
// network learns an O(1) factor that carries over between sizes, and for a
// constant-coefficient stencil the scale reduces to 1 / sqrt(a_jj).
// Features f_i: degree, a_ii, sum / mean / min / max / std of |a_ij| (j != i)
// and a_ii / sum, each z-scored over the rows of A.
// Loss over pairs (r_s, e_s) = (A u_s, u_s) from the solver's basis: the
// mean squared sine of the angle between M r_s and e_s (independent of the
// scale of M r_s, as the inner Krylov space is):
//   L = (1/S) sum_s [1 - a_s^2 / (b_s c_s)],  q = G^T G r, a = <q, e>,
//   b = ||q||^2, c = ||e||^2;
//   dL/dG(i,j) = sum_s (y_i z_j + (G z)_i r_j),  y = G r,
//   z = (-2 a / (b c) e + 2 a^2 / (b^2 c) q) / S  (a sampled dense-dense
//   product on the pattern).
// All reductions are fixed-order (per-block partials, then one block), so a
// training step is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include <algorithm>

#include "common.h"

namespace trplk {

namespace {

constexpr int NF = MLP_NF;
constexpr int NIN = MLP_NIN;
constexpr int NH = MLP_NH;
constexpr int NP = MLP_NPARAM;
constexpr int OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH;

int g1(int64_t n) { return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))); }

// ---------------------------------------------------------------- features
__global__ void k_raw_features(int n, const int* rowptr, const int* col, const double* val,
                               double* F) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double d = 0.0, s = 0.0, mn = 0.0, mx = 0.0;
    int deg = 0;
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j) {
      if (col[j] == i) {
        d = val[j];
        continue;
      }
      const double o = fabs(val[j]);
      s += o;
      mn = deg ? fmin(mn, o) : o;
      mx = deg ? fmax(mx, o) : o;
      ++deg;
    }
    double sd = 0.0, mean = 0.0;
    if (deg) {
      mean = s / deg;
      double q = 0.0;
      for (int j = rowptr[i]; j < rowptr[i + 1]; ++j)
        if (col[j] != i) {
          const double t = fabs(val[j]) - mean;
          q += t * t;
        }
      sd = sqrt(q / deg);
    }
    double* f = F + static_cast<int64_t>(i) * NF;
    f[0] = deg;
    f[1] = d;
    f[2] = s;
    f[3] = mean;
    f[4] = mn;
    f[5] = mx;
    f[6] = sd;
    f[7] = deg ? d / s : 0.0;
  }
}

// per-block sums of F (pass 0) or of (F - mu)^2 (pass 1), one row of NF per block
__global__ __launch_bounds__(256) void k_feat_moments(int n, const double* F, const double* mu,
                                                      double* part) {
  __shared__ double red[256][NF];
  double acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double v = F[static_cast<int64_t>(i) * NF + f];
      if (mu) {
        const double t = v - mu[f];
        acc[f] += t * t;
      } else {
        acc[f] += v;
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) red[threadIdx.x][f] = acc[f];
  __syncthreads();
  if (threadIdx.x < NF) {
    double t = 0.0;
    for (int q = 0; q < 256; ++q) t += red[q][threadIdx.x];
    part[blockIdx.x * NF + threadIdx.x] = t;
  }
}

__global__ void k_feat_stat(int nblk, int n, const double* part, double* out, int sqrt_mode) {
  const int f = threadIdx.x;
  if (f >= NF) return;
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += part[b * NF + f];
  t /= n;
  if (sqrt_mode) {
    t = sqrt(t);
    if (t == 0.0) t = 1.0;
  }
  out[f] = t;
}

__global__ void k_feat_norm(int n, const double* F, const double* mu, const double* sd, float* Fz) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
       t < static_cast<int64_t>(n) * NF; t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int f = static_cast<int>(t % NF);
    Fz[t] = static_cast<float>((F[t] - mu[f]) / sd[f]);
  }
}

// ------------------------------------------------------------ tril pattern
__global__ void k_tril_count(int n, const int* rowptr, const int* col, int* cnt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int c = 0;
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j) c += col[j] <= i;
    cnt[i] = c;
  }
}

__global__ void k_tril_fill(int n, const int* rowptr, const int* col, const double* val,
                            const int* lrow, int* lcol, int* lr, double* lval) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int o = lrow[i];
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j)
      if (col[j] <= i) {
        lcol[o] = col[j];
        lr[o] = i;
        lval[o] = val[j];
        ++o;
      }
  }
}

// ------------------------------------------------------------------- MLP
__device__ __forceinline__ void load_params(const float* P, float* sP) {
  for (int t = threadIdx.x; t < NP; t += blockDim.x) sP[t] = P[t];
  __syncthreads();
}

__device__ __forceinline__ void make_input(const float* Fz, const double* dinv, int i, int j,
                                           double aij, float* x) {
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    x[f] = Fz[static_cast<int64_t>(i) * NF + f];
    x[NF + f] = Fz[static_cast<int64_t>(j) * NF + f];
  }
  x[2 * NF] = static_cast<float>(fabs(aij) * sqrt(dinv[i] * dinv[j]));
}

__global__ __launch_bounds__(256) void k_mlp_forward(int64_t nnz, const int* lr, const int* lc,
                                                     const double* lval, const float* Fz,
                                                     const double* dinv, const double* cbar,
                                                     const float* P, double* gval, float* oval) {
  __shared__ float sP[NP];
  load_params(P, sP);
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < nnz;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int i = lr[e], j = lc[e];
    float x[NIN];
    make_input(Fz, dinv, i, j, lval[e], x);
    float o = sP[OFF_B2];
    for (int k = 0; k < NH; ++k) {
      float pre = sP[OFF_B1 + k];
#pragma unroll
      for (int f = 0; f < NIN; ++f) pre += sP[k * NIN + f] * x[f];
      o += sP[OFF_W2 + k] * fmaxf(pre, 0.0f);
    }
    if (oval) oval[e] = o;
    const double od = static_cast<double>(o);
    gval[e] = i == j ? exp(od) * sqrt(dinv[j]) : -od * lval[e] * dinv[j] * sqrt(dinv[i]) / *cbar;
  }
}

// -------------------------------------------------- pair algebra (float64)
// Y = M X for a CSR M and row-major n x S blocks (S <= 64): a wavefront per
// row, lane s owns column s.  With E: Y = M X - E.
__global__ __launch_bounds__(256) void k_spmm(int n, int S, const int* rowptr, const int* col,
                                              const double* val, const double* X, const double* E,
                                              double* Y) {
  const int lane = threadIdx.x & 63;
  for (int i = (blockIdx.x * blockDim.x + threadIdx.x) / 64; i < n;
       i += (gridDim.x * blockDim.x) / 64) {
    if (lane >= S) continue;
    double t = 0.0;
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j)
      t += val[j] * X[static_cast<int64_t>(col[j]) * S + lane];
    if (E) t -= E[static_cast<int64_t>(i) * S + lane];
    Y[static_cast<int64_t>(i) * S + lane] = t;
  }
}

// per-block partials of a_s = <Q_s, E_s> (slot s) and b_s = ||Q_s||^2
// (slot 64 + s): lane s of each wavefront owns column s
__global__ __launch_bounds__(256) void k_pair_dots(int n, int S, const double* Q, const double* E,
                                                   double* part) {
  __shared__ double ra[4][64], rb[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x / 64;
  double a = 0.0, b = 0.0;
  if (lane < S)
    for (int i = blockIdx.x * 4 + wv; i < n; i += gridDim.x * 4) {
      const double q = Q[static_cast<int64_t>(i) * S + lane];
      a += q * E[static_cast<int64_t>(i) * S + lane];
      b += q * q;
    }
  ra[wv][lane] = a;
  rb[wv][lane] = b;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int t = threadIdx.x;
    part[blockIdx.x * 128 + t] = ra[0][t] + ra[1][t] + ra[2][t] + ra[3][t];
    part[blockIdx.x * 128 + 64 + t] = rb[0][t] + rb[1][t] + rb[2][t] + rb[3][t];
  }
}

// coefficients of z and the loss; coef[s] = -2a/(bcS), coef[64+s] = 2a^2/(b^2 c S)
__global__ void k_pair_coef(int nblk, int S, const double* part, const double* en, double* coef,
                            double* loss) {
  __shared__ double ls[64];
  const int s = threadIdx.x;
  double l = 0.0;
  if (s < S) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < nblk; ++q) {
      a += part[q * 128 + s];
      b += part[q * 128 + 64 + s];
    }
    const double c = en[s];
    coef[s] = -2.0 * a / (b * c * S);
    coef[64 + s] = 2.0 * a * a / (b * b * c * S);
    l = 1.0 - a * a / (b * c);
  }
  if (s < 64) ls[s] = l;
  __syncthreads();
  if (s == 0) {
    double t = 0.0;
    for (int q = 0; q < S; ++q) t += ls[q];
    *loss = t / S;
  }
}

__global__ void k_make_z(int n, int S, const double* coef, const double* E, const double* Q,
                         double* Z) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
       t < static_cast<int64_t>(n) * S; t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int s = static_cast<int>(t % S);
    Z[t] = coef[s] * E[t] + coef[64 + s] * Q[t];
  }
}

// column norms of a row-major n x S block: per-block partials [S]
// column norms of a row-major n x S block: lane s of each wavefront sums
// column s over the wavefront's rows; per-block partials [64]
__global__ __launch_bounds__(256) void k_colnorm_part(int n, int S, const double* E, double* part) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x / 64;
  double acc = 0.0;
  if (lane < S)
    for (int i = blockIdx.x * 4 + wv; i < n; i += gridDim.x * 4) {
      const double v = E[static_cast<int64_t>(i) * S + lane];
      acc += v * v;
    }
  red[wv][lane] = acc;
  __syncthreads();
  if (threadIdx.x < 64)
    part[blockIdx.x * 64 + threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] +
                                          red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ void k_colnorms(int nblk, int S, const double* part, double* en) {
  const int s = threadIdx.x;
  if (s >= S) return;
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += part[b * 64 + s];
  en[s] = t;
}

// dL/do_e: sampled products on the pattern, then the chain rule through
// G = exp(o)/sqrt(a_ii) (diagonal) or -o a_ij / (cbar a_jj sqrt(a_ii))
__global__ __launch_bounds__(256) void k_sddmm(int64_t nnz, int S, const int* lr, const int* lc,
                                               const double* lval, const double* gval,
                                               const double* dinv, const double* cbar,
                                               const double* Y, const double* Z, const double* Uz,
                                               const double* R, float* dout) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < nnz;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int i = lr[e], j = lc[e];
    const double* yi = Y + static_cast<int64_t>(i) * S;
    const double* ui = Uz + static_cast<int64_t>(i) * S;
    const double* zj = Z + static_cast<int64_t>(j) * S;
    const double* rj = R + static_cast<int64_t>(j) * S;
    double g = 0.0;
    for (int s = 0; s < S; ++s) g += yi[s] * zj[s] + ui[s] * rj[s];
    const double dodg = (i == j) ? gval[e] : -lval[e] * dinv[j] * sqrt(dinv[i]) / *cbar;
    dout[e] = static_cast<float>(g * dodg);
  }
}

// MLP backward: per-block partial gradients of sum_e do_e * o_e.  A block
// takes chunks of BWC nonzeros: forward recompute into LDS, then thread t
// owns parameters t, t + 256, ... and sums their contributions over the
// chunk in a fixed order; partials accumulate in registers across chunks.
constexpr int BWC = 128;
constexpr int PPT = (NP + 255) / 256;  // parameters per thread

__global__ __launch_bounds__(256) void k_mlp_backward(int64_t nnz, const int* lr, const int* lc,
                                                      const double* lval, const float* Fz,
                                                      const double* dinv, const float* P,
                                                      const float* dout, double* part) {
  __shared__ float sP[NP];
  __shared__ float sx[BWC][NIN + 1];
  __shared__ float sdp[BWC][NH + 1];  // dpre
  __shared__ float sh[BWC][NH + 1];   // h
  __shared__ float sdo[BWC];
  load_params(P, sP);
  double acc[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) acc[q] = 0.0;
  const int64_t nchunk = (nnz + BWC - 1) / BWC;
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int64_t e0 = ch * BWC;
    // forward recompute: threads 0..BWC-1 one nonzero each
    if (threadIdx.x < BWC) {
      const int64_t e = e0 + threadIdx.x;
      float x[NIN];
      float d = 0.0f;
      if (e < nnz) {
        make_input(Fz, dinv, lr[e], lc[e], lval[e], x);
        d = dout[e];
      } else {
#pragma unroll
        for (int f = 0; f < NIN; ++f) x[f] = 0.0f;
      }
#pragma unroll
      for (int f = 0; f < NIN; ++f) sx[threadIdx.x][f] = x[f];
      sdo[threadIdx.x] = d;
      for (int k = 0; k < NH; ++k) {
        float pre = sP[OFF_B1 + k];
#pragma unroll
        for (int f = 0; f < NIN; ++f) pre += sP[k * NIN + f] * x[f];
        const bool on = pre > 0.0f;
        sh[threadIdx.x][k] = on ? pre : 0.0f;
        sdp[threadIdx.x][k] = on ? d * sP[OFF_W2 + k] : 0.0f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = threadIdx.x + 256 * q;
      if (p >= NP) continue;
      float t = 0.0f;
      if (p < OFF_B1) {
        const int k = p / NIN, f = p % NIN;
        for (int c = 0; c < BWC; ++c) t += sdp[c][k] * sx[c][f];
      } else if (p < OFF_W2) {
        const int k = p - OFF_B1;
        for (int c = 0; c < BWC; ++c) t += sdp[c][k];
      } else if (p < OFF_B2) {
        const int k = p - OFF_W2;
        for (int c = 0; c < BWC; ++c) t += sdo[c] * sh[c][k];
      } else {
        for (int c = 0; c < BWC; ++c) t += sdo[c];
      }
      acc[q] += static_cast<double>(t);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + 256 * q;
    if (p < NP) part[static_cast<int64_t>(blockIdx.x) * NP + p] = acc[q];
  }
}

__global__ void k_param_sum(int nblk, const double* part, double* grad) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NP; p += gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += part[static_cast<int64_t>(b) * NP + p];
    grad[p] = t;
  }
}

__global__ void k_sum_small(int nblk, const double* part, double* out) {
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += part[b];
  *out = t;
}

// Adam (Kingma and Ba), float32 parameters and moments, step count t >= 1
// Adam (Kingma and Ba, Algorithm 1) in float32.  The weights 1 - beta and
// the bias corrections 1 - beta^t come from the host, formed in float64 and
// rounded once: 1 - 0.999f in float32 is 0.99998713e-3, 1.3e-5 off the
// method's 1e-3.
__global__ void k_adam(float* P, float* m, float* v, const double* grad, float lr, float b1,
                       float om1, float b2, float om2, float c1, float c2, float eps) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NP; p += gridDim.x * blockDim.x) {
    const float g = static_cast<float>(grad[p]);
    m[p] = b1 * m[p] + om1 * g;
    v[p] = b2 * v[p] + om2 * (g * g);
    const float mh = m[p] / c1, vh = v[p] / c2;
    P[p] -= lr * mh / (sqrtf(vh) + eps);
  }
}

__global__ void k_to_rowmajor(int n, int S, const double* Xc, int64_t ldx, double* Xr) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
       t < static_cast<int64_t>(n) * S; t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = t / S, s = t % S;
    Xr[t] = Xc[s * ldx + i];
  }
}

}  // namespace

// ------------------------------------------------------------- launchers --
hipError_t mlp_features(int n, const int* rowptr, const int* col, const double* val, double* F,
                        float* Fz, double* scratch, hipStream_t s) {
  const int nb = std::min(g1(n), 1024);
  double* part = scratch;              // nb * NF
  double* mu = scratch + nb * NF;      // NF
  double* sd = mu + NF;                // NF
  hipLaunchKernelGGL(k_raw_features, dim3(g1(n)), dim3(256), 0, s, n, rowptr, col, val, F);
  hipLaunchKernelGGL(k_feat_moments, dim3(nb), dim3(256), 0, s, n, F, nullptr, part);
  hipLaunchKernelGGL(k_feat_stat, dim3(1), dim3(64), 0, s, nb, n, part, mu, 0);
  hipLaunchKernelGGL(k_feat_moments, dim3(nb), dim3(256), 0, s, n, F, mu, part);
  hipLaunchKernelGGL(k_feat_stat, dim3(1), dim3(64), 0, s, nb, n, part, sd, 1);
  hipLaunchKernelGGL(k_feat_norm, dim3(g1(static_cast<int64_t>(n) * NF)), dim3(256), 0, s, n, F,
                     mu, sd, Fz);
  return hipGetLastError();
}

int mlp_scratch_doubles() { return 1024 * NF + 2 * NF; }

hipError_t tril_count(int n, const int* rowptr, const int* col, int* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_tril_count, dim3(g1(n)), dim3(256), 0, s, n, rowptr, col, cnt);
  return hipGetLastError();
}

hipError_t tril_fill(int n, const int* rowptr, const int* col, const double* val, const int* lrow,
                     int* lcol, int* lr, double* lval, hipStream_t s) {
  hipLaunchKernelGGL(k_tril_fill, dim3(g1(n)), dim3(256), 0, s, n, rowptr, col, val, lrow, lcol, lr,
                     lval);
  return hipGetLastError();
}

hipError_t mlp_forward(int64_t nnz, const int* lr, const int* lc, const double* lval,
                       const float* Fz, const double* dinv, const double* cbar, const float* P,
                       double* gval, float* oval, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(g1(nnz)), dim3(256), 0, s, nnz, lr, lc, lval, Fz, dinv,
                     cbar, P, gval, oval);
  return hipGetLastError();
}

// cbar: mean of |a_ij| sqrt(dinv_i dinv_j) over the strictly lower entries
// (1 when there are none), two fixed-order stages
constexpr int CB_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_coupling_part(int64_t nnz, const int* lr, const int* lc,
                                                       const double* lval, const double* dinv,
                                                       double* part) {
  double sum = 0.0, cnt = 0.0;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < nnz;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int i = lr[e], j = lc[e];
    if (i != j) {
      sum += fabs(lval[e]) * sqrt(dinv[i] * dinv[j]);
      cnt += 1.0;
    }
  }
  __shared__ double red[2][256 / WAVE];
  sum = wave_sum(sum);
  cnt = wave_sum(cnt);
  if ((threadIdx.x & (WAVE - 1)) == 0) {
    red[0][threadIdx.x / WAVE] = sum;
    red[1][threadIdx.x / WAVE] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 256 / WAVE; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

__global__ void k_coupling_final(int nblk, const double* part, double* cbar) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nblk; ++k) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  cbar[0] = (b > 0.0 && a > 0.0) ? a / b : 1.0;
}

hipError_t coupling_scale(int64_t nnz, const int* lr, const int* lc, const double* lval,
                          const double* dinv, double* part, double* cbar, hipStream_t s) {
  hipLaunchKernelGGL(k_coupling_part, dim3(CB_BLOCKS), dim3(256), 0, s, nnz, lr, lc, lval, dinv,
                     part);
  hipLaunchKernelGGL(k_coupling_final, dim3(1), dim3(64), 0, s, CB_BLOCKS, part, cbar);
  return hipGetLastError();
}

int learn_blocks() { return 512; }

// One evaluation of the loss and its gradient with respect to the MLP
// parameters.  Rr, Er: row-major n x S pairs; G given by (Lrow, lc, gval)
// and its transpose by (Trow, Tcol, perm) with values gval[perm].
hipError_t learn_loss_grad(const LearnArgs& a, hipStream_t s) {
  const int S = a.S;
  const int nb = learn_blocks();
  const dim3 gs(g1(static_cast<int64_t>(a.n) * 64)), bs(256);
  // y = G r, q = G^T y
  hipLaunchKernelGGL(k_spmm, gs, bs, 0, s, a.n, S, a.Lrow, a.lc, a.gval, a.Rr, nullptr, a.Y);
  hipLaunchKernelGGL(k_spmm, gs, bs, 0, s, a.n, S, a.Trow, a.Tcol, a.gvalT, a.Y, nullptr, a.Q);
  hipLaunchKernelGGL(k_pair_dots, dim3(256), dim3(256), 0, s, a.n, S, a.Q, a.Er, a.part);
  hipLaunchKernelGGL(k_pair_coef, dim3(1), dim3(64), 0, s, 256, S, a.part, a.en, a.coef, a.loss);
  hipLaunchKernelGGL(k_make_z, dim3(g1(static_cast<int64_t>(a.n) * S)), bs, 0, s, a.n, S, a.coef,
                     a.Er, a.Q, a.Z);
  hipLaunchKernelGGL(k_spmm, gs, bs, 0, s, a.n, S, a.Lrow, a.lc, a.gval, a.Z, nullptr, a.Uz);
  hipLaunchKernelGGL(k_sddmm, dim3(g1(a.nnz)), bs, 0, s, a.nnz, S, a.lr, a.lc, a.lval, a.gval,
                     a.dinv, a.cbar, a.Y,
                     a.Z, a.Uz, a.Rr, a.dout);
  hipLaunchKernelGGL(k_mlp_backward, dim3(nb), bs, 0, s, a.nnz, a.lr, a.lc, a.lval, a.Fz, a.dinv,
                     a.P, a.dout, a.part);
  hipLaunchKernelGGL(k_param_sum, dim3(8), bs, 0, s, nb, a.part, a.grad);
  return hipGetLastError();
}

hipError_t learn_colnorms(int n, int S, const double* Er, double* part, double* en, hipStream_t s) {
  const int nb = 256;
  hipLaunchKernelGGL(k_colnorm_part, dim3(nb), dim3(256), 0, s, n, S, Er, part);
  hipLaunchKernelGGL(k_colnorms, dim3(1), dim3(64), 0, s, nb, S, part, en);
  return hipGetLastError();
}

hipError_t gather_values(int64_t nnz, const double* src, const double* permd, double* dst, hipStream_t s);

hipError_t adam_step(float* P, float* m, float* v, const double* grad, int t, float lr,
                     hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  hipLaunchKernelGGL(k_adam, dim3(8), dim3(256), 0, s, P, m, v, grad, lr, static_cast<float>(b1),
                     static_cast<float>(1.0 - b1), static_cast<float>(b2), static_cast<float>(1.0 - b2),
                     static_cast<float>(1.0 - std::pow(b1, t)), static_cast<float>(1.0 - std::pow(b2, t)),
                     1e-8f);
  return hipGetLastError();
}

hipError_t to_rowmajor(int n, int S, const double* Xc, int64_t ldx, double* Xr, hipStream_t s) {
  hipLaunchKernelGGL(k_to_rowmajor, dim3(g1(static_cast<int64_t>(n) * S)), dim3(256), 0, s, n, S,
                     Xc, ldx, Xr);
  return hipGetLastError();
}

namespace {
__global__ void k_gather(int64_t nnz, const double* src, const double* permd, double* dst) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < nnz;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[t] = src[static_cast<int64_t>(permd[t])];
}
__global__ void k_iota(int64_t nnz, double* x) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < nnz;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[t] = static_cast<double>(t);
}
}  // namespace

hipError_t gather_values(int64_t nnz, const double* src, const double* permd, double* dst,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(g1(nnz)), dim3(256), 0, s, nnz, src, permd, dst);
  return hipGetLastError();
}

hipError_t iota_values(int64_t nnz, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(g1(nnz)), dim3(256), 0, s, nnz, x);
  return hipGetLastError();
}

}  // namespace trplk
