// Learned smooth vector: a two-layer message-passing network over the
// matrix graph that predicts log w, where w is the algebraically smooth
// vector that drives the matching weights (Sec. 3.1 leaves its source open;
// targets come from the method's own relaxation).  Activations and the
// weights of the dense products are stored in bfloat16; products accumulate
// in binary32.  The dense layers run on MFMA (v_mfma_f32_16x16x16 bf16).
//
// Node features (8): 1, log(a_ii)/4, s_i/a_ii (s_i = sum_{j!=i}|a_ij|), two
// l1-Jacobi sweeps on A w = 0 from ones, log(max/min off-diagonal |a_ij|)/4,
// (#off-diagonals)/6, 0.  Aggregation (Ahat X)_i = sum_{j!=i} |a_ij| X_j / s_i.
//   h1 = ReLU([X | Ahat X] W1 + b1), h2 = ReLU([h1 | Ahat h1] W2 + b2),
//   y = h2 wh + bh.
// Parameters, flat: W1 (16x32 row-major), b1 (32), W2 (64x32), b2 (32),
// wh (32), bh (1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <cstdlib>
#include <cstdio>
#include <mutex>
#include <vector>

#include "amg_internal.hpp"

namespace amg {
namespace {

constexpr int kF0 = 8, kHid = 32;
constexpr int oW1 = 0, ob1 = 2 * kF0 * kHid, oW2 = ob1 + kHid, ob2 = oW2 + 2 * kHid * kHid,
              owh = ob2 + kHid, obh = owh + kHid, kNP = obh + 1;
static_assert(kNP == AMG_MPNN_NPARAMS, "parameter count");
constexpr int kRowsDW = 1024;   // rows per workgroup in the weight-gradient reductions

typedef unsigned short bf16;
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

inline dim3 grid_for(int64_t n, int block = kBlock) {
  return dim3(static_cast<unsigned>(std::max<int64_t>(1, (n + block - 1) / block)));
}

// binary32 -> bfloat16, round to nearest, ties to even
__device__ __forceinline__ bf16 f2bf(float f) {
  unsigned b = __float_as_uint(f);
  b = b + 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<bf16>(b >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(static_cast<unsigned>(h) << 16); }

// ------------------------------------------------------------- features
// A row's CSR entries, eight at a time with every load of a batch issued
// before the first use; f(k, col, val) in CSR order.
template <class F>
__device__ __forceinline__ void csr_row_batched(int kb, int ke, const int *__restrict__ ci,
                                                const double *__restrict__ v, F f) {
  for (int k0 = kb; k0 < ke; k0 += 8) {
    int c[8];
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < ke) {
        c[u] = ci[k0 + u];
        a[u] = v[k0 + u];
      }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < ke) f(k0 + u, c[u], a[u]);
  }
}

// Features 0-3 and 5-7 of row i (feature 4, the second sweep, is k_feat2's),
// stored as one 16-byte row with a zero in place of feature 4.
__global__ void k_feat1(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                        const double *__restrict__ v, bf16 *__restrict__ X, float *__restrict__ s_out,
                        double *__restrict__ w1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0, s = 0.0, l1 = 0.0, ax = 0.0, mx = 0.0, mn = INFINITY;
  int noff = 0;
  csr_row_batched(rp[i], rp[i + 1], ci, v, [&](int, int c, double a) {
    l1 = l1 + fabs(a);
    ax = ax + a;
    if (c == i) {
      d = a;
      return;
    }
    s = s + fabs(a);
    mx = fmax(mx, fabs(a));
    mn = fmin(mn, fabs(a));
    ++noff;
  });
  const double w = 1.0 - (1.0 / l1) * ax;
  w1[i] = w;
  s_out[i] = static_cast<float>(s);
  bf16 x[kF0];
  x[0] = f2bf(1.0f);
  x[1] = f2bf(static_cast<float>(log(d) / 4.0));
  x[2] = f2bf(static_cast<float>(s / d));
  x[3] = f2bf(static_cast<float>(w));
  x[4] = 0;
  x[5] = f2bf(noff > 0 ? static_cast<float>(log(mx / mn) / 4.0) : 0.0f);
  x[6] = f2bf(static_cast<float>(noff / 6.0));
  x[7] = f2bf(0.0f);
  uint4 o;
  __builtin_memcpy(&o, x, sizeof(o));
  *reinterpret_cast<uint4 *>(X + static_cast<int64_t>(i) * kF0) = o;
}

__global__ void k_feat2(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                        const double *__restrict__ v, const double *__restrict__ w1,
                        bf16 *__restrict__ X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double l1 = 0.0, ax = 0.0;
  const int kb = rp[i], ke = rp[i + 1];
  for (int k0 = kb; k0 < ke; k0 += 8) {
    int c[8];
    double a[8], wv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < ke) {
        c[u] = ci[k0 + u];
        a[u] = v[k0 + u];
      }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < ke) wv[u] = w1[c[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < ke) {
        l1 = l1 + fabs(a[u]);
        ax = ax + a[u] * wv[u];
      }
  }
  X[static_cast<int64_t>(i) * kF0 + 4] = f2bf(static_cast<float>(w1[i] - (1.0 / l1) * ax));
}

// ----------------------------------------------------------- aggregation
// out_i = sum_{j != i} |a_ij| H_j / s_i, binary32 fold in CSR order.  A lane
// handles 8 features (one 16-byte load of a bfloat16 row piece), F / 8 lanes
// per row; the row's entries are taken 8 at a time with all loads of a batch
// in flight together.
template <int F>
__global__ void __launch_bounds__(kBlock) k_agg(int n, const int *__restrict__ rp,
                                                const int *__restrict__ ci,
                                                const double *__restrict__ v,
                                                const float *__restrict__ s,
                                                const bf16 *__restrict__ H, bf16 *__restrict__ out) {
  static_assert(F % 8 == 0, "8 features per lane");
  constexpr int LPR = F / 8;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int i = static_cast<int>(t / LPR), f0 = static_cast<int>(t % LPR) * 8;
  if (i >= n) return;
  float acc[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) acc[e] = 0.0f;
  const int kb = rp[i], ke = rp[i + 1];
  for (int k0 = kb; k0 < ke; k0 += 8) {
    int jv[8];
    float av[8];
    uint4 hv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      jv[u] = -1;
      if (k0 + u < ke) {
        jv[u] = ci[k0 + u];
        av[u] = static_cast<float>(fabs(v[k0 + u]));
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (jv[u] >= 0 && jv[u] != i)
        hv[u] = *reinterpret_cast<const uint4 *>(H + static_cast<int64_t>(jv[u]) * F + f0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (jv[u] >= 0 && jv[u] != i) {
        const unsigned w[4] = {hv[u].x, hv[u].y, hv[u].z, hv[u].w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bf16 h = static_cast<bf16>((w[e / 2] >> (16 * (e % 2))) & 0xFFFFu);
          acc[e] = acc[e] + av[u] * bf2f(h);
        }
      }
    }
  }
  const float si = s[i];
  unsigned o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int e = 0; e < 8; ++e)
    o[e / 2] |= static_cast<unsigned>(f2bf(si > 0.0f ? acc[e] / si : 0.0f)) << (16 * (e % 2));
  *reinterpret_cast<uint4 *>(out + static_cast<int64_t>(i) * F + f0) = make_uint4(o[0], o[1], o[2], o[3]);
}

// (Ahat^T D)_i added to acc: sum_{j != i} (|a_ij| / s_j) D_j (symmetric pattern and values).
template <int F>
__global__ void __launch_bounds__(kBlock) k_agg_t_add(int n, const int *__restrict__ rp,
                                                      const int *__restrict__ ci,
                                                      const double *__restrict__ v,
                                                      const float *__restrict__ s,
                                                      const float *__restrict__ D,
                                                      float *__restrict__ acc_io) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int i = static_cast<int>(t / F), f = static_cast<int>(t % F);
  if (i >= n) return;
  float acc = 0.0f;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = ci[k];
    if (j == i) continue;
    const float sj = s[j];
    if (sj > 0.0f) acc = acc + (static_cast<float>(fabs(v[k])) / sj) * D[static_cast<int64_t>(j) * F + f];
  }
  acc_io[t] = acc_io[t] + acc;
}

// ------------------------------------------------------- dense layer (MFMA)
// H = ReLU([Ua | Ub] W + b) for 16-row tiles, one wavefront per tile.
// Wt is W transposed (32 x K, bfloat16).  MFMA 16x16x16 (bf16 in, f32 acc):
// lane l supplies A[row l%16][k 4(l/16)..+3], B[k 4(l/16)..+3][col l%16] and
// receives D[row 4(l/16)+i][col l%16], i = 0..3.
constexpr int kDenseTiles = 4;   // 16-row tiles per wavefront (their loads in flight together)

template <int K>
__global__ void __launch_bounds__(kBlock) k_dense(int n, const bf16 *__restrict__ Ua,
                                                  const bf16 *__restrict__ Ub,
                                                  const bf16 *__restrict__ Wt,
                                                  const float *__restrict__ b,
                                                  bf16 *__restrict__ H) {
  constexpr int FH = K / 2;
  // the wavefront's output tiles (16 x 32 each), written out as whole 64-byte rows
  __shared__ __attribute__((aligned(16))) bf16 tile[kBlock / kWave][kDenseTiles * 16 * kHid];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int r0 = (blockIdx.x * (kBlock / kWave) + wv) * (16 * kDenseTiles);
  if (r0 >= n) return;
  const int kq = 4 * (lane >> 4);
  short4v a[kDenseTiles][K / 16];
#pragma unroll
  for (int t = 0; t < kDenseTiles; ++t) {
    const int arow = r0 + 16 * t + (lane & 15);
#pragma unroll
    for (int kc = 0; kc < K / 16; ++kc) {
      const int k = kc * 16 + kq;
      a[t][kc] = short4v{0, 0, 0, 0};
      if (arow < n) {
        const bf16 *src = (k < FH) ? Ua + static_cast<int64_t>(arow) * FH + k
                                   : Ub + static_cast<int64_t>(arow) * FH + (k - FH);
        a[t][kc] = *reinterpret_cast<const short4v *>(src);
      }
    }
  }
  bf16 *T = tile[wv];
#pragma unroll
  for (int ct = 0; ct < kHid / 16; ++ct) {
    short4v bb[K / 16];
#pragma unroll
    for (int kc = 0; kc < K / 16; ++kc)
      bb[kc] = *reinterpret_cast<const short4v *>(Wt + static_cast<int64_t>(ct * 16 + (lane & 15)) * K +
                                                  kc * 16 + kq);
    const int col = ct * 16 + (lane & 15);
    const float bias = b[col];
#pragma unroll
    for (int t = 0; t < kDenseTiles; ++t) {
      float4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < K / 16; ++kc)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t][kc], bb[kc], acc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) T[(16 * t + kq + q) * kHid + col] = f2bf(fmaxf(acc[q] + bias, 0.0f));
    }
  }
  __builtin_amdgcn_wave_barrier();   // a wavefront's LDS accesses complete in issue order
#pragma unroll
  for (int t = 0; t < kDenseTiles; ++t) {
    const int lr = 16 * t + (lane >> 2);
    if (r0 + lr < n)
      *reinterpret_cast<uint4 *>(H + static_cast<int64_t>(r0 + lr) * kHid + 8 * (lane & 3)) =
          *reinterpret_cast<const uint4 *>(T + lr * kHid + 8 * (lane & 3));
  }
}

// y_i = sum_c h_ic wh_c + bh (binary32, c ascending); w_i = exp(y_i)
__global__ void k_head(int n, const bf16 *__restrict__ H, const float *__restrict__ theta,
                       float *__restrict__ y, double *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.0f;
  const bf16 *h = H + static_cast<int64_t>(i) * kHid;
  for (int c = 0; c < kHid; ++c) acc = acc + bf2f(h[c]) * theta[owh + c];
  acc = acc + theta[obh];
  y[i] = acc;
  if (w) w[i] = exp(static_cast<double>(acc));
}

// --------------------------------------------------------------- backward
// loss partials (sum of squared differences) and dy = 2 (y - log w*) / n
__global__ void k_loss(int n, const float *__restrict__ y, const double *__restrict__ wt,
                       float *__restrict__ dy, float *__restrict__ part) {
  __shared__ float red[kBlock];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float e2 = 0.0f;
  if (i < n) {
    const float d = y[i] - static_cast<float>(log(wt[i]));
    dy[i] = 2.0f * d / static_cast<float>(n);
    e2 = d * d;
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// G_ic = dy_i wh_c [h_ic > 0]
__global__ void k_head_bwd(int n, const bf16 *__restrict__ H, const float *__restrict__ dy,
                           const float *__restrict__ theta, float *__restrict__ G) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= static_cast<int64_t>(n) * kHid) return;
  const int i = static_cast<int>(t / kHid), c = static_cast<int>(t % kHid);
  G[t] = (bf2f(H[t]) > 0.0f) ? dy[i] * theta[owh + c] : 0.0f;
}

// Per-workgroup partial of U^T G over kRowsDW rows: part[blk][k][c], k < K
// (U = [Ua | Ub], bfloat16), plus the column sums of G (bias gradient) in
// part[blk][K][c] and, when hy is given, the head gradient: sum_i h_ic dy_i in
// part[blk][K+1][c] and sum_i dy_i in part[blk][K+2][0].
template <int K>
__global__ void __launch_bounds__(kBlock) k_dw(int n, const bf16 *__restrict__ Ua,
                                               const bf16 *__restrict__ Ub,
                                               const float *__restrict__ G,
                                               const bf16 *__restrict__ hy_h,
                                               const float *__restrict__ hy_dy,
                                               float *__restrict__ part) {
  constexpr int FH = K / 2, NP = K * kHid, PPT = NP / kBlock, TR = 32;
  __shared__ float su[TR][K];
  __shared__ float sg[TR][kHid];
  __shared__ float sdy[TR];
  const int r_begin = blockIdx.x * kRowsDW;
  const int r_end = min(n, r_begin + kRowsDW);
  float acc[PPT > 0 ? PPT : 1];
#pragma unroll
  for (int q = 0; q < (PPT > 0 ? PPT : 1); ++q) acc[q] = 0.0f;
  float bsum = 0.0f, hsum = 0.0f, dsum = 0.0f;   // thread c < 32: bias / head sums
  for (int t0 = r_begin; t0 < r_end; t0 += TR) {
    for (int e = threadIdx.x; e < TR * K; e += kBlock) {
      const int r = e / K, k = e % K, row = t0 + r;
      float u = 0.0f;
      if (row < r_end) u = bf2f(k < FH ? Ua[static_cast<int64_t>(row) * FH + k] : Ub[static_cast<int64_t>(row) * FH + k - FH]);
      su[r][k] = u;
    }
    for (int e = threadIdx.x; e < TR * kHid; e += kBlock) {
      const int r = e / kHid, c = e % kHid, row = t0 + r;
      sg[r][c] = (row < r_end) ? G[static_cast<int64_t>(row) * kHid + c] : 0.0f;
    }
    if (hy_dy && threadIdx.x < TR) {
      const int row = t0 + threadIdx.x;
      sdy[threadIdx.x] = (row < r_end) ? hy_dy[row] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = threadIdx.x + q * kBlock, k = p / kHid, c = p % kHid;
      float a = acc[q];
      for (int r = 0; r < TR; ++r) a = a + su[r][k] * sg[r][c];
      acc[q] = a;
    }
    if (threadIdx.x < kHid) {
      const int c = threadIdx.x;
      for (int r = 0; r < TR; ++r) bsum = bsum + sg[r][c];
      if (hy_dy) {
        for (int r = 0; r < TR; ++r) {
          const int row = t0 + r;
          const float hv = (row < r_end) ? bf2f(hy_h[static_cast<int64_t>(row) * kHid + c]) : 0.0f;
          hsum = hsum + hv * sdy[r];
        }
        if (c == 0)
          for (int r = 0; r < TR; ++r) dsum = dsum + sdy[r];
      }
    }
    __syncthreads();
  }
  float *out = part + static_cast<int64_t>(blockIdx.x) * (K + 3) * kHid;
#pragma unroll
  for (int q = 0; q < PPT; ++q) out[threadIdx.x + q * kBlock] = acc[q];
  if (threadIdx.x < kHid) {
    out[K * kHid + threadIdx.x] = bsum;
    out[(K + 1) * kHid + threadIdx.x] = hsum;
    out[(K + 2) * kHid + threadIdx.x] = (threadIdx.x == 0) ? dsum : 0.0f;
  }
}

// Fold the per-workgroup partials in workgroup order: out[m] = sum_b part[b][m].
__global__ void k_fold_parts(int nb, int m, const float *__restrict__ part, float *__restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  float acc = 0.0f;
  for (int b = 0; b < nb; ++b) acc = acc + part[static_cast<int64_t>(b) * m + e];
  out[e] = acc;
}

// dU = G W^T for W = bf16-rounded W2 (64 x 32): dself (k < 32), dneigh (k >= 32)
__global__ void k_dx2(int n, const float *__restrict__ G, const bf16 *__restrict__ Wt2,
                      float *__restrict__ dself, float *__restrict__ dneigh) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= static_cast<int64_t>(n) * 2 * kHid) return;
  const int i = static_cast<int>(t / (2 * kHid)), k = static_cast<int>(t % (2 * kHid));
  const float *g = G + static_cast<int64_t>(i) * kHid;
  float acc = 0.0f;
  for (int c = 0; c < kHid; ++c) acc = acc + g[c] * bf2f(Wt2[c * 2 * kHid + k]);
  if (k < kHid) dself[static_cast<int64_t>(i) * kHid + k] = acc;
  else dneigh[static_cast<int64_t>(i) * kHid + k - kHid] = acc;
}

// G1 = dh1 [h1 > 0]
__global__ void k_relu_bwd(int64_t m, const float *__restrict__ dh, const bf16 *__restrict__ H,
                           float *__restrict__ G) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t < m) G[t] = (bf2f(H[t]) > 0.0f) ? dh[t] : 0.0f;
}

// gradient vector from the folded partials (layout of the parameters)
__global__ void k_gather_grad(const float *__restrict__ f1, const float *__restrict__ f2,
                              float *__restrict__ g) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNP) return;
  float v;
  if (e < ob1) v = f1[e];                                        // W1: [k][c], k < 16
  else if (e < oW2) v = f1[16 * kHid + (e - ob1)];                // b1
  else if (e < ob2) v = f2[e - oW2];                              // W2: [k][c], k < 64
  else if (e < owh) v = f2[64 * kHid + (e - ob2)];                // b2
  else if (e < obh) v = f2[65 * kHid + (e - owh)];                // wh
  else v = f2[66 * kHid];                                         // bh
  g[e] = v;
}

// Adam (Kingma & Ba), then the bfloat16 transposed weight copies.
__global__ void k_adam(float *__restrict__ theta, const float *__restrict__ g,
                       float *__restrict__ m1, float *__restrict__ m2, float lr, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNP) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gg = g[e];
  const float a = b1 * m1[e] + (1.0f - b1) * gg;
  const float b = b2 * m2[e] + (1.0f - b2) * gg * gg;
  m1[e] = a;
  m2[e] = b;
  theta[e] = theta[e] - lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ void k_pack_weights(const float *__restrict__ theta, bf16 *__restrict__ Wt1,
                               bf16 *__restrict__ Wt2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < 2 * kF0 * kHid) {           // W1[k][c] -> Wt1[c][k]
    const int k = e / kHid, c = e % kHid;
    Wt1[c * 2 * kF0 + k] = f2bf(theta[oW1 + e]);
  }
  if (e < 2 * kHid * kHid) {          // W2[k][c] -> Wt2[c][k]
    const int k = e / kHid, c = e % kHid;
    Wt2[c * 2 * kHid + k] = f2bf(theta[oW2 + e]);
  }
}

}  // namespace
}  // namespace amg

// =================================================================== model
struct amg_mpnn {
  hipStream_t stream = nullptr;
  int own_stream = 0;
  int cap = 0;                      // rows the forward buffers hold
  int cap_train = 0;                // rows the backward buffers hold
  int step = 0;
  amg::dvec<float> theta, m1, m2, grad;
  amg::dvec<unsigned short> Wt1, Wt2;
  amg::dvec<unsigned short> X0, N0, h1, N1, h2;
  amg::dvec<float> s, y, dy, G2, dself, dneigh, G1, part, f1, f2;
  amg::dvec<double> w1;
};

namespace amg {
namespace {

void mpnn_alloc_params(amg_mpnn *m) {
  m->theta.alloc(kNP); m->m1.alloc(kNP); m->m2.alloc(kNP); m->grad.alloc(kNP);
  m->Wt1.alloc(2 * kF0 * kHid); m->Wt2.alloc(2 * kHid * kHid);
  m->f1.alloc(19 * kHid); m->f2.alloc(67 * kHid);
}

// Parameters (NULL: zeros) to the device, packed weights, Adam moments
// cleared; synchronises m->stream.
void mpnn_load_params(amg_mpnn *m, const float *params) {
  std::vector<float> init(kNP, 0.0f);
  if (params) std::memcpy(init.data(), params, sizeof(float) * kNP);
  for (float x : init)
    if (!std::isfinite(x)) fail(AMG_ERR_NONFINITE, "non-finite network parameter");
  AMG_HIP(hipMemcpyAsync(m->theta.p, init.data(), sizeof(float) * kNP, hipMemcpyHostToDevice, m->stream));
  AMG_HIP(hipMemsetAsync(m->m1.p, 0, sizeof(float) * kNP, m->stream));
  AMG_HIP(hipMemsetAsync(m->m2.p, 0, sizeof(float) * kNP, m->stream));
  hipLaunchKernelGGL(k_pack_weights, grid_for(2 * kHid * kHid), dim3(kBlock), 0, m->stream, m->theta.p,
                     m->Wt1.p, m->Wt2.p);
  AMG_LAUNCH_CHECK();
  AMG_HIP(hipStreamSynchronize(m->stream));
}

}  // namespace
}  // namespace amg


namespace amg {
namespace {

// Forward buffers (features, activations, prediction) for n rows; the
// backward pass's buffers only when training.
void mpnn_reserve(amg_mpnn *m, int n) {
  if (n <= m->cap) return;
  const size_t N = static_cast<size_t>(n);
  m->X0.alloc(N * kF0); m->N0.alloc(N * kF0);
  m->h1.alloc(N * kHid); m->N1.alloc(N * kHid); m->h2.alloc(N * kHid);
  m->s.alloc(N); m->y.alloc(N); m->w1.alloc(N);
  m->cap = n;
}

void mpnn_reserve_train(amg_mpnn *m, int n) {
  if (n <= m->cap_train) return;
  const size_t N = static_cast<size_t>(n);
  m->dy.alloc(N);
  m->G2.alloc(N * kHid); m->dself.alloc(N * kHid); m->dneigh.alloc(N * kHid); m->G1.alloc(N * kHid);
  const size_t nb = (N + kRowsDW - 1) / kRowsDW;
  m->part.alloc(std::max<size_t>(nb * (64 + 3) * kHid, (N + kBlock - 1) / kBlock));
  m->cap_train = n;
}

void check_csr(const amg_csr *A) {
  if (!A || A->n <= 0 || !A->row_ptr || !A->col_idx || !A->val || !A->on_device)
    fail(AMG_ERR_INVALID, "the network takes a device CSR");
}

void mpnn_forward(amg_mpnn *m, const amg_csr *A, double *w_out) {
  hipStream_t s = m->stream;
  const int n = A->n;
  mpnn_reserve(m, n);
  const int *rp = A->row_ptr, *ci = A->col_idx;
  const double *v = A->val;
  hipLaunchKernelGGL(k_feat1, grid_for(n), dim3(kBlock), 0, s, n, rp, ci, v, m->X0.p, m->s.p, m->w1.p);
  hipLaunchKernelGGL(k_feat2, grid_for(n), dim3(kBlock), 0, s, n, rp, ci, v, m->w1.p, m->X0.p);
  hipLaunchKernelGGL(k_agg<kF0>, grid_for(static_cast<int64_t>(n) * (kF0 / 8)), dim3(kBlock), 0, s, n, rp, ci,
                     v, m->s.p, m->X0.p, m->N0.p);
  const dim3 gd = grid_for(ceil_div(n, 16 * kDenseTiles), kBlock / kWave);
  hipLaunchKernelGGL(k_dense<2 * kF0>, gd, dim3(kBlock), 0, s, n, m->X0.p, m->N0.p, m->Wt1.p,
                     m->theta.p + ob1, m->h1.p);
  hipLaunchKernelGGL(k_agg<kHid>, grid_for(static_cast<int64_t>(n) * (kHid / 8)), dim3(kBlock), 0, s, n, rp,
                     ci, v, m->s.p, m->h1.p, m->N1.p);
  hipLaunchKernelGGL(k_dense<2 * kHid>, gd, dim3(kBlock), 0, s, n, m->h1.p, m->N1.p, m->Wt2.p,
                     m->theta.p + ob2, m->h2.p);
  hipLaunchKernelGGL(k_head, grid_for(n), dim3(kBlock), 0, s, n, m->h2.p, m->theta.p, m->y.p, w_out);
  AMG_LAUNCH_CHECK();
}

float mpnn_train(amg_mpnn *m, const amg_csr *A, const double *wt, float lr, float *grad_host) {
  hipStream_t s = m->stream;
  const int n = A->n;
  mpnn_reserve_train(m, n);
  mpnn_forward(m, A, nullptr);
  const int *rp = A->row_ptr, *ci = A->col_idx;
  const double *v = A->val;
  const int nbl = ceil_div(n, kBlock);
  hipLaunchKernelGGL(k_loss, dim3(nbl), dim3(kBlock), 0, s, n, m->y.p, wt, m->dy.p, m->part.p);
  dvec<float> lsum(1);
  hipLaunchKernelGGL(k_fold_parts, dim3(1), dim3(1), 0, s, nbl, 1, m->part.p, lsum.p);
  float loss = 0.0f;
  AMG_HIP(hipMemcpyAsync(&loss, lsum.p, sizeof(float), hipMemcpyDeviceToHost, s));
  const int64_t nh = static_cast<int64_t>(n) * kHid;
  hipLaunchKernelGGL(k_head_bwd, grid_for(nh), dim3(kBlock), 0, s, n, m->h2.p, m->dy.p, m->theta.p, m->G2.p);
  const int nbd = ceil_div(n, kRowsDW);
  // layer 2: dW2, db2, dwh, dbh
  hipLaunchKernelGGL(k_dw<2 * kHid>, dim3(nbd), dim3(kBlock), 0, s, n, m->h1.p, m->N1.p, m->G2.p,
                     m->h2.p, m->dy.p, m->part.p);
  hipLaunchKernelGGL(k_fold_parts, grid_for(67 * kHid), dim3(kBlock), 0, s, nbd, 67 * kHid, m->part.p,
                     m->f2.p);
  // back through layer 2 into h1
  hipLaunchKernelGGL(k_dx2, grid_for(2 * nh), dim3(kBlock), 0, s, n, m->G2.p, m->Wt2.p, m->dself.p,
                     m->dneigh.p);
  hipLaunchKernelGGL(k_agg_t_add<kHid>, grid_for(nh), dim3(kBlock), 0, s, n, rp, ci, v, m->s.p,
                     m->dneigh.p, m->dself.p);
  hipLaunchKernelGGL(k_relu_bwd, grid_for(nh), dim3(kBlock), 0, s, nh, m->dself.p, m->h1.p, m->G1.p);
  // layer 1: dW1, db1
  hipLaunchKernelGGL(k_dw<2 * kF0>, dim3(nbd), dim3(kBlock), 0, s, n, m->X0.p, m->N0.p, m->G1.p,
                     nullptr, nullptr, m->part.p);
  hipLaunchKernelGGL(k_fold_parts, grid_for(19 * kHid), dim3(kBlock), 0, s, nbd, 19 * kHid, m->part.p,
                     m->f1.p);
  hipLaunchKernelGGL(k_gather_grad, grid_for(kNP), dim3(kBlock), 0, s, m->f1.p, m->f2.p, m->grad.p);
  if (grad_host) AMG_HIP(hipMemcpyAsync(grad_host, m->grad.p, sizeof(float) * kNP, hipMemcpyDeviceToHost, s));
  if (lr > 0.0f) {
    m->step += 1;
    const float c1 = 1.0f - powf(0.9f, static_cast<float>(m->step));
    const float c2 = 1.0f - powf(0.999f, static_cast<float>(m->step));
    hipLaunchKernelGGL(k_adam, grid_for(kNP), dim3(kBlock), 0, s, m->theta.p, m->grad.p, m->m1.p, m->m2.p,
                       lr, c1, c2);
    hipLaunchKernelGGL(k_pack_weights, grid_for(2 * kHid * kHid), dim3(kBlock), 0, s, m->theta.p,
                       m->Wt1.p, m->Wt2.p);
  }
  AMG_LAUNCH_CHECK();
  AMG_HIP(hipStreamSynchronize(s));
  return loss / static_cast<float>(n);
}

}  // namespace
}  // namespace amg

namespace amg {

// Model file: the numbers of the first [...] after a "params" key, or the
// file's first numbers when it has no such key; white space and commas
// separate them.  Exactly AMG_MPNN_NPARAMS are taken; fewer, or text that is
// not a number before they are complete, is a failure.
bool mpnn_read_params_file(const char *path, float *out) {
  if (!path || !out) return false;
  std::FILE *f = std::fopen(path, "rb");
  if (!f) return false;
  std::string text;
  char buf[1 << 16];
  for (size_t got; (got = std::fread(buf, 1, sizeof(buf), f)) > 0;) text.append(buf, got);
  const bool read_ok = !std::ferror(f);
  std::fclose(f);
  if (!read_ok) return false;
  size_t pos = 0;
  const size_t key = text.find("\"params\"");
  if (key != std::string::npos) {
    pos = text.find('[', key);
    if (pos == std::string::npos) return false;
    ++pos;
  }
  const char *p = text.c_str() + pos;
  for (int i = 0; i < AMG_MPNN_NPARAMS; ++i) {
    while (*p == ' ' || *p == ',' || *p == '\n' || *p == '\r' || *p == '\t') ++p;
    char *end = nullptr;
    const double v = std::strtod(p, &end);
    if (end == p) return false;
    out[i] = static_cast<float>(v);
    p = end;
  }
  return true;
}

// The network inside amg_setup (AMG_SMOOTH_LEARNED): one network per device,
// kept for the life of the process, so that a setup does not allocate and
// free the forward buffers (about 224 bytes per row) each time; they grow
// to the largest n seen.  Setups on one device take turns (mutex); the
// work runs on the setup's stream s and is finished when this returns.
int mpnn_predict_for_setup(const float *params, const amg_csr *A, double *w_out, hipStream_t s) {
  struct Cache {
    std::mutex mu;
    amg_mpnn *m = nullptr;
  };
  static Cache cache[kMaxDevices];
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(AMG_ERR_DEVICE, "device index out of range");
  Cache &c = cache[dev];
  std::lock_guard<std::mutex> lock(c.mu);
  NoPool no_pool;   // the buffers outlive this setup and its stream
  return api_guarded([&] {
    if (!c.m) {
      amg_mpnn *m = new amg_mpnn();
      m->stream = s;
      try {
        mpnn_alloc_params(m);
      } catch (...) {
        delete m;
        throw;
      }
      c.m = m;
    }
    amg_mpnn *m = c.m;
    m->stream = s;
    mpnn_load_params(m, params);
    check_csr(A);
    mpnn_forward(m, A, w_out);
    AMG_HIP(hipStreamSynchronize(s));
    m->stream = nullptr;
    return AMG_OK;
  });
}

}  // namespace amg

extern "C" {

int amg_mpnn_read_params(const char *path, float *params) {
  if (!path || !params) return amg::api_set_error(AMG_ERR_INVALID, "NULL argument");
  if (!amg::mpnn_read_params_file(path, params))
    return amg::api_set_error(AMG_ERR_MODEL, std::string("cannot read network parameters from ") + path);
  return AMG_OK;
}

int amg_mpnn_create(const float *params, void *stream, amg_mpnn **out) {
  if (out) *out = nullptr;
  if (!out) return amg::api_set_error(AMG_ERR_INVALID, "NULL out");
  amg_mpnn *m = new (std::nothrow) amg_mpnn();
  if (!m) return amg::api_set_error(AMG_ERR_NOMEM, "host allocation failed");
  if (stream) {
    m->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreate(&m->stream) != hipSuccess) {
      delete m;
      return amg::api_set_error(AMG_ERR_DEVICE, "hipStreamCreate failed");
    }
    m->own_stream = 1;
  }
  const int st = amg::api_guarded([&] {
    amg::mpnn_alloc_params(m);
    amg::mpnn_load_params(m, params);
    return AMG_OK;
  });
  if (st != AMG_OK) {
    std::string msg = amg::api_last_error();
    amg_mpnn_destroy(m);
    amg::api_set_error(st, msg);
    return st;
  }
  *out = m;
  return AMG_OK;
}

int amg_mpnn_get_params(const amg_mpnn *m, float *params) {
  if (!m || !params) return amg::api_set_error(AMG_ERR_INVALID, "NULL argument");
  return amg::api_guarded([&] {
    AMG_HIP(hipMemcpyAsync(params, m->theta.p, sizeof(float) * AMG_MPNN_NPARAMS, hipMemcpyDeviceToHost, m->stream));
    AMG_HIP(hipStreamSynchronize(m->stream));
    return AMG_OK;
  });
}

int amg_mpnn_features(amg_mpnn *m, const amg_csr *A, float *X_host) {
  if (!m || !X_host) return amg::api_set_error(AMG_ERR_INVALID, "NULL argument");
  return amg::api_guarded([&] {
    using namespace amg;
    check_csr(A);
    mpnn_forward(m, A, nullptr);
    const size_t cnt = static_cast<size_t>(A->n) * kF0;
    std::vector<unsigned short> tmp(cnt);
    AMG_HIP(hipMemcpyAsync(tmp.data(), m->X0.p, sizeof(unsigned short) * cnt, hipMemcpyDeviceToHost, m->stream));
    AMG_HIP(hipStreamSynchronize(m->stream));
    for (size_t e = 0; e < cnt; ++e) {
      const unsigned u = static_cast<unsigned>(tmp[e]) << 16;
      std::memcpy(&X_host[e], &u, sizeof(float));
    }
    return AMG_OK;
  });
}

int amg_mpnn_predict(amg_mpnn *m, const amg_csr *A, double *w_out, float *y_host) {
  if (!m || (!w_out && !y_host)) return amg::api_set_error(AMG_ERR_INVALID, "NULL argument");
  return amg::api_guarded([&] {
    using namespace amg;
    check_csr(A);
    mpnn_forward(m, A, w_out);
    if (y_host) AMG_HIP(hipMemcpyAsync(y_host, m->y.p, sizeof(float) * A->n, hipMemcpyDeviceToHost, m->stream));
    AMG_HIP(hipStreamSynchronize(m->stream));
    return AMG_OK;
  });
}

int amg_mpnn_train_step(amg_mpnn *m, const amg_csr *A, const double *w_target, float lr,
                        float *loss_out, float *grad_host) {
  if (!m || !w_target || !loss_out || !(lr >= 0.0f)) return amg::api_set_error(AMG_ERR_INVALID, "bad argument");
  return amg::api_guarded([&] {
    amg::check_csr(A);
    *loss_out = amg::mpnn_train(m, A, w_target, lr, grad_host);
    return std::isfinite(*loss_out) ? AMG_OK : amg::api_set_error(AMG_ERR_NONFINITE, "non-finite loss");
  });
}

void amg_mpnn_destroy(amg_mpnn *m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  hipStream_t s = m->stream;
  const int own = m->own_stream;
  delete m;
  if (own) (void)hipStreamDestroy(s);
}

}  // extern "C"
