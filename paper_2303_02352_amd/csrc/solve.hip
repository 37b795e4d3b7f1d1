// Solve phase: V-cycle (Alg. 2) and flexible PCG (Alg. 1) on the GPU.
//
// Matrices are read in the SELL-64 layout (one wavefront of rows per slice,
// one row per lane, entries in CSR order), so every row sum is a left fold
// in CSR order: SpMV, sweeps, residuals, restriction and prolongation give
// the same bits as a sequential evaluation.  Only the three PCG dot products
// and the residual norm are tree reductions (fixed order, so repeatable).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "amg_internal.hpp"

namespace amg {

namespace {

inline dim3 grid_for(int64_t n, int block = kBlock) {
  return dim3(static_cast<unsigned>(std::max<int64_t>(1, (n + block - 1) / block)));
}

// ------------------------------------------------------ SELL row kernels
// Row r of slice s: slots sptr[s] + k*64 + lane, k < width(s).
template <class T>
__device__ __forceinline__ void sell_row(const int *__restrict__ sptr, const int *__restrict__ col,
                                         const T *__restrict__ val, const T *__restrict__ x, int r,
                                         T &sum, T &l1) {
  const int s = r >> 6, lane = r & 63;
  const int b = sptr[s], width = (sptr[s + 1] - b) >> 6;
  const int *cp = col + b + lane;
  const T *vp = val + b + lane;
  T acc = T(0), m = T(0);
  int k = 0;
  for (; k + 4 <= width; k += 4) {
    const int c0 = ld_stream(cp + (k + 0) * 64), c1 = ld_stream(cp + (k + 1) * 64);
    const int c2 = ld_stream(cp + (k + 2) * 64), c3 = ld_stream(cp + (k + 3) * 64);
    const T a0 = ld_stream(vp + (k + 0) * 64), a1 = ld_stream(vp + (k + 1) * 64);
    const T a2 = ld_stream(vp + (k + 2) * 64), a3 = ld_stream(vp + (k + 3) * 64);
    const T x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
    acc = acc + a0 * x0; m = m + fabs(a0);
    acc = acc + a1 * x1; m = m + fabs(a1);
    acc = acc + a2 * x2; m = m + fabs(a2);
    acc = acc + a3 * x3; m = m + fabs(a3);
  }
  for (; k < width; ++k) {
    const int c = ld_stream(cp + k * 64);
    const T a = ld_stream(vp + k * 64);
    acc = acc + a * x[c];
    m = m + fabs(a);
  }
  sum = acc;
  l1 = m;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_spmv(int n, const int *__restrict__ sptr,
                                                 const int *__restrict__ col,
                                                 const T *__restrict__ val, const T *__restrict__ x,
                                                 T *__restrict__ y) {
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r >= n) return;
  T s, m;
  sell_row(sptr, col, val, x, r, s, m);
  y[r] = s;
}

// l1-Jacobi sweep: xn = x + dinv * (r - A x), dinv = 1 / sum_j |a_ij| taken
// from the streamed row (same fold as the stored diagonal would use).
template <class T>
__global__ void __launch_bounds__(kBlock) k_sweep(int n, const int *__restrict__ sptr,
                                                  const int *__restrict__ col,
                                                  const T *__restrict__ val,
                                                  const T *__restrict__ rhs,
                                                  const T *__restrict__ x, T *__restrict__ xn) {
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r >= n) return;
  T s, m;
  sell_row(sptr, col, val, x, r, s, m);
  const T di = T(1) / m;
  xn[r] = x[r] + di * (rhs[r] - s);
}

// First sweep from x = 0: x = dinv * r.
template <class T>
__global__ void __launch_bounds__(kBlock) k_sweep_first(int n, const T *__restrict__ dinv,
                                                        const T *__restrict__ rhs,
                                                        T *__restrict__ x) {
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r < n) x[r] = dinv[r] * rhs[r];
}

// Residual + restriction fused per aggregate:
// rc[I] = sum over members i of I (ascending) of p_i (r_i - (A x)_i).
template <class T>
__global__ void __launch_bounds__(kBlock) k_restrict(int nc, const int *__restrict__ mptr,
                                                     const int *__restrict__ mem,
                                                     const T *__restrict__ pval,
                                                     const int *__restrict__ sptr,
                                                     const int *__restrict__ col,
                                                     const T *__restrict__ val,
                                                     const T *__restrict__ rhs,
                                                     const T *__restrict__ x, T *__restrict__ rc) {
  const int I = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (I >= nc) return;
  T acc = T(0);
  for (int q = mptr[I]; q < mptr[I + 1]; ++q) {
    const int i = mem[q];
    T s, m;
    sell_row(sptr, col, val, x, i, s, m);
    acc = acc + pval[i] * (rhs[i] - s);
  }
  rc[I] = acc;
}

// x_i += p_i * e[agg_i]
template <class T>
__global__ void __launch_bounds__(kBlock) k_prolong(int n, const int *__restrict__ agg,
                                                    const T *__restrict__ pval,
                                                    const T *__restrict__ e, T *__restrict__ x) {
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r < n) x[r] = x[r] + pval[r] * e[agg[r]];
}

template <class T>
__global__ void k_zero(int n, T *x) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) x[r] = T(0);
}

__global__ void k_f2d(int n, const float *a, double *b) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = static_cast<double>(a[r]);
}

// ---------------------------------------------------- coarsest direct solve
// One wavefront: L y = r by columns (k ascending per row), then L^T x = y by
// columns (k descending per row): the same folds as row-oriented substitution.
template <class TI, class TO>
__global__ void __launch_bounds__(kWave) k_chol_solve(int n, const double *__restrict__ Lcm,
                                                      const double *__restrict__ Lrm,
                                                      const TI *__restrict__ rin,
                                                      TO *__restrict__ xout) {
  extern __shared__ double sh[];
  double *s = sh;        // running right-hand side
  double *y = sh + n;    // solution of the current triangle
  for (int i = threadIdx.x; i < n; i += kWave) s[i] = static_cast<double>(rin[i]);
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double yj = s[j] / Lcm[static_cast<int64_t>(j) * n + j];
    if (threadIdx.x == 0) y[j] = yj;
    for (int i = j + 1 + threadIdx.x; i < n; i += kWave)
      s[i] = s[i] - Lcm[static_cast<int64_t>(j) * n + i] * yj;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += kWave) s[i] = y[i];
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double xj = s[j] / Lrm[static_cast<int64_t>(j) * n + j];
    if (threadIdx.x == 0) y[j] = xj;
    for (int i = threadIdx.x; i < j; i += kWave)
      s[i] = s[i] - Lrm[static_cast<int64_t>(j) * n + i] * xj;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += kWave) xout[i] = static_cast<TO>(y[i]);
}

// ----------------------------------------------------------- PCG kernels
// Row chunking shared by the reduction kernels: G <= 2048 workgroups, each
// owns a contiguous run of rows (multiple of 256) and writes one partial per
// quantity; the last workgroup to finish folds the partials in index order.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int wid = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[wid] = v;
  __syncthreads();
  double t = red[0];
  for (int q = 1; q < kBlock / kWave; ++q) t = t + red[q];
  return t;
}

// Returns true in every thread of the last workgroup to arrive.
__device__ __forceinline__ bool arrive_last(unsigned *counter) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (last) __threadfence();
  return last;
}

__device__ __forceinline__ double fold_partials(const double *part, int np, int stride_off,
                                                double *red) {
  double t = 0.0;
  for (int q = threadIdx.x; q < np; q += kBlock) t = t + part[q * 3 + stride_off];
  return block_sum(t, red);
}

// r = b - A u; ||r||^2.  Last block: nr0, threshold rtol * nr0, reset state.
__global__ void __launch_bounds__(kBlock) k_pcg_init(int n, int rpb, const int *__restrict__ sptr,
                                                     const int *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ b,
                                                     const double *__restrict__ u,
                                                     double *__restrict__ r, double *part,
                                                     unsigned *counter, Scalars *sc, double rtol) {
  __shared__ double red[kBlock / kWave];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * rpb, r1 = min(n, r0 + rpb);
  double rr = 0.0;
  for (int row = r0 + threadIdx.x; row < r1; row += kBlock) {
    double s, m;
    sell_row(sptr, col, val, u, row, s, m);
    const double ri = b[row] - s;
    r[row] = ri;
    rr = rr + ri * ri;
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) part[lb * 3] = rr;
  if (!arrive_last(counter)) return;
  const double tot = fold_partials(part, gridDim.x, 0, red);
  if (threadIdx.x == 0) {
    const double nr0 = sqrt(tot);
    sc->nr0 = nr0;
    sc->rr = tot;
    sc->thr = rtol * nr0;
    sc->rho = 1.0;
    sc->c = 0.0;
    sc->a = 0.0;
    sc->it = 0;
    sc->status = isfinite(nr0) ? 0 : AMG_ERR_NONFINITE;
    sc->done = (nr0 == 0.0 || !isfinite(nr0)) ? 1 : 0;
    *counter = 0u;
  }
}

// v = A w; alpha = w.r, beta = w.v, gamma = w.q.  Last block: rho, c, a (Alg. 1).
__global__ void __launch_bounds__(kBlock) k_pcg_spmv_dots(
    int n, int rpb, const int *__restrict__ sptr, const int *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ w, const double *__restrict__ r,
    const double *__restrict__ q, double *__restrict__ v, double *part, unsigned *counter,
    Scalars *sc) {
  __shared__ double red[kBlock / kWave];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * rpb, r1 = min(n, r0 + rpb);
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int row = r0 + threadIdx.x; row < r1; row += kBlock) {
    double s, m;
    sell_row(sptr, col, val, w, row, s, m);
    v[row] = s;
    const double wi = w[row];
    al = al + wi * r[row];
    be = be + wi * s;
    ga = ga + wi * q[row];
  }
  al = block_sum(al, red);
  be = block_sum(be, red);
  ga = block_sum(ga, red);
  if (threadIdx.x == 0) {
    part[lb * 3 + 0] = al;
    part[lb * 3 + 1] = be;
    part[lb * 3 + 2] = ga;
  }
  if (!arrive_last(counter)) return;
  const double A = fold_partials(part, gridDim.x, 0, red);
  const double B = fold_partials(part, gridDim.x, 1, red);
  const double G = fold_partials(part, gridDim.x, 2, red);
  if (threadIdx.x == 0) {
    const double rho_prev = sc->rho;
    const double rho = B - (G * G) / rho_prev;
    sc->alpha = A;
    sc->beta = B;
    sc->gamma = G;
    if (!isfinite(rho) || !isfinite(A)) {
      sc->status = AMG_ERR_NONFINITE;
      sc->done = 1;
    } else if (!(rho > 0.0)) {
      sc->status = AMG_ERR_NOT_SPD;
      sc->done = 1;
    }
    sc->c = G / rho_prev;
    sc->a = A / rho;
    sc->rho = rho;
    *counter = 0u;
  }
}

// d = w - c d; u = u + a d; q = v - c q; r = r - a q; ||r||^2.
// Last block: convergence test ||r|| <= rtol ||r_0|| (Sec. 5).
__global__ void __launch_bounds__(kBlock) k_pcg_update(int n, int rpb, const double *__restrict__ w,
                                                       const double *__restrict__ v,
                                                       double *__restrict__ d,
                                                       double *__restrict__ u,
                                                       double *__restrict__ q,
                                                       double *__restrict__ r, double *part,
                                                       unsigned *counter, Scalars *sc) {
  __shared__ double red[kBlock / kWave];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * rpb, r1 = min(n, r0 + rpb);
  const double c = sc->c, a = sc->a;
  double rr = 0.0;
  for (int i = r0 + threadIdx.x; i < r1; i += kBlock) {
    const double di = w[i] - c * d[i];
    d[i] = di;
    u[i] = u[i] + a * di;
    const double qi = v[i] - c * q[i];
    q[i] = qi;
    const double ri = r[i] - a * qi;
    r[i] = ri;
    rr = rr + ri * ri;
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) part[lb * 3] = rr;
  if (!arrive_last(counter)) return;
  const double tot = fold_partials(part, gridDim.x, 0, red);
  if (threadIdx.x == 0) {
    const double nr = sqrt(tot);
    sc->rr = tot;
    sc->it = sc->it + 1;
    if (nr <= sc->thr) sc->done = 1;
    else if (!isfinite(nr)) { sc->status = AMG_ERR_NONFINITE; sc->done = 1; }
    *counter = 0u;
  }
}

// ------------------------------------------------------------ V-cycle
template <class T> const T *vals(const Sell &S);
template <> const double *vals<double>(const Sell &S) { return S.val.p; }
template <> const float *vals<float>(const Sell &S) { return S.valf.p; }
template <class T> const T *dinv_of(const Level &L);
template <> const double *dinv_of<double>(const Level &L) { return L.dinv.p; }
template <> const float *dinv_of<float>(const Level &L) { return L.dinvf.p; }
template <class T> const T *pval_of(const Level &L);
template <> const double *pval_of<double>(const Level &L) { return L.pval.p; }
template <> const float *pval_of<float>(const Level &L) { return L.pvalf.p; }
template <class T> T *rbuf(Level &L);
template <> double *rbuf<double>(Level &L) { return L.r.p; }
template <> float *rbuf<float>(Level &L) { return L.rf.p; }
template <class T> T *xbuf(Level &L);
template <> double *xbuf<double>(Level &L) { return L.x.p; }
template <> float *xbuf<float>(Level &L) { return L.xf.p; }
template <class T> T *tbuf(Level &L);
template <> double *tbuf<double>(Level &L) { return L.t.p; }
template <> float *tbuf<float>(Level &L) { return L.tf.p; }

template <class T>
void launch_sweep(const Level &L, const T *rhs, const T *x, T *xn, hipStream_t s) {
  const int n = L.A.n;
  hipLaunchKernelGGL(k_sweep<T>, grid_for(n), dim3(kBlock), 0, s, n, L.S.sptr.p, L.S.col.p,
                     vals<T>(L.S), rhs, x, xn);
}

// Level k of the V-cycle in precision T; result lands in `out`.
template <class T>
void vcycle_level(amg_hierarchy *h, int k, const T *rhs, T *out) {
  hipStream_t s = h->stream;
  Level &L = h->L[k];
  const int n = L.A.n;
  const int nl = static_cast<int>(h->L.size());
  const amg_params &P = h->p;
  if (k == nl - 1) {
    if (h->coarse_dense) {
      const size_t shm = sizeof(double) * 2 * n;
      hipLaunchKernelGGL((k_chol_solve<T, T>), dim3(1), dim3(kWave), shm, s, n, h->Lc.p, h->LcT.p,
                         rhs, out);
    } else {
      const int sw = P.coarse_sweeps;
      T *A = (sw - 1) % 2 == 0 ? out : tbuf<T>(L);
      T *B = (A == out) ? tbuf<T>(L) : out;
      hipLaunchKernelGGL(k_sweep_first<T>, grid_for(n), dim3(kBlock), 0, s, n, dinv_of<T>(L), rhs, A);
      for (int q = 1; q < sw; ++q) { launch_sweep<T>(L, rhs, A, B, s); std::swap(A, B); }
    }
    return;
  }
  const int swaps = (P.pre_sweeps > 0 ? P.pre_sweeps - 1 : 0) + P.post_sweeps;
  T *A = (swaps % 2 == 0) ? out : tbuf<T>(L);
  T *B = (A == out) ? tbuf<T>(L) : out;
  if (P.pre_sweeps == 0) {
    hipLaunchKernelGGL(k_zero<T>, grid_for(n), dim3(kBlock), 0, s, n, A);
  } else {
    hipLaunchKernelGGL(k_sweep_first<T>, grid_for(n), dim3(kBlock), 0, s, n, dinv_of<T>(L), rhs, A);
    for (int q = 1; q < P.pre_sweeps; ++q) { launch_sweep<T>(L, rhs, A, B, s); std::swap(A, B); }
  }
  Level &C = h->L[k + 1];
  hipLaunchKernelGGL(k_restrict<T>, grid_for(L.nc), dim3(kBlock), 0, s, L.nc, L.mptr.p, L.mem.p,
                     pval_of<T>(L), L.S.sptr.p, L.S.col.p, vals<T>(L.S), rhs, A, rbuf<T>(C));
  vcycle_level<T>(h, k + 1, rbuf<T>(C), xbuf<T>(C));
  hipLaunchKernelGGL(k_prolong<T>, grid_for(n), dim3(kBlock), 0, s, n, L.agg.p, pval_of<T>(L),
                     xbuf<T>(C), A);
  for (int q = 0; q < P.post_sweeps; ++q) { launch_sweep<T>(L, rhs, A, B, s); std::swap(A, B); }
}

// Mixed precision (R: binary32 V-cycle, binary64 outer iteration): r is
// rounded to binary32 on entry, the whole cycle (coarsest solve excepted,
// which converts to binary64 inside its kernel) runs in binary32, and the
// result is widened back to binary64.
__global__ void k_d2f_vec(int n, const double *a, float *b) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = static_cast<float>(a[r]);
}

void vcycle_mixed(amg_hierarchy *h, const double *r, double *z) {
  hipStream_t s = h->stream;
  Level &L = h->L[0];
  const int n = L.A.n;
  if (h->L.size() == 1) {   // single level: the direct solve in binary64
    vcycle_level<double>(h, 0, r, z);
    return;
  }
  hipLaunchKernelGGL(k_d2f_vec, grid_for(n), dim3(kBlock), 0, s, n, r, L.rf.p);
  vcycle_level<float>(h, 0, L.rf.p, L.xf.p);
  hipLaunchKernelGGL(k_f2d, grid_for(n), dim3(kBlock), 0, s, n, L.xf.p, z);
}

}  // namespace

// ----------------------------------------------------------------- API
void alloc_solve_buffers(amg_hierarchy *h) {
  const bool mixed = (h->p.precision == AMG_PREC_MIXED);
  for (size_t k = 0; k < h->L.size(); ++k) {
    Level &L = h->L[k];
    const int n = L.A.n;
    L.r.alloc(n);
    L.x.alloc(n);
    L.t.alloc(n);
    if (mixed) {
      L.rf.alloc(n);
      L.xf.alloc(n);
      L.tf.alloc(n);
    }
  }
  const int n = h->L[0].A.n;
  h->u.alloc(n); h->r.alloc(n); h->w.alloc(n); h->v.alloc(n); h->d.alloc(n); h->q.alloc(n);
  h->partials.alloc(kMaxDotBlocks * 3);
  h->counter.alloc(1);
  h->sc.alloc(1);
  AMG_HIP(hipMemsetAsync(h->counter.p, 0, sizeof(unsigned), h->stream));
  if (!h->sc_host) AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->sc_host), sizeof(Scalars)));
}

void enqueue_vcycle(amg_hierarchy *h, const double *r, double *z) {
  const int n = h->L[0].A.n;
  if (!h->p.precond) {
    AMG_HIP(hipMemcpyAsync(z, r, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    return;
  }
  if (h->p.precision == AMG_PREC_MIXED) vcycle_mixed(h, r, z);
  else vcycle_level<double>(h, 0, r, z);
  AMG_LAUNCH_CHECK();
}

void enqueue_spmv(amg_hierarchy *h, int k, const double *x, double *y) {
  const Level &L = h->L[k];
  hipLaunchKernelGGL(k_spmv<double>, grid_for(L.A.n), dim3(kBlock), 0, h->stream, L.A.n, L.S.sptr.p,
                     L.S.col.p, L.S.val.p, x, y);
  AMG_LAUNCH_CHECK();
}

void enqueue_sweep(amg_hierarchy *h, int k, const double *r, const double *x, double *xn) {
  launch_sweep<double>(h->L[k], r, x, xn, h->stream);
  AMG_LAUNCH_CHECK();
}

namespace {
int dot_blocks(int n) { return std::min(kMaxDotBlocks, std::max(1, ceil_div(n, kBlock))); }
int rows_per_block(int n, int G) { return ceil_div(ceil_div(n, G), kBlock) * kBlock; }

void enqueue_iteration(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  const Level &L0 = h->L[0];
  const int n = L0.A.n, G = dot_blocks(n), rpb = rows_per_block(n, G);
  enqueue_vcycle(h, h->r.p, h->w.p);
  hipLaunchKernelGGL(k_pcg_spmv_dots, dim3(G), dim3(kBlock), 0, s, n, rpb, L0.S.sptr.p, L0.S.col.p,
                     L0.S.val.p, h->w.p, h->r.p, h->q.p, h->v.p, h->partials.p, h->counter.p,
                     h->sc.p);
  hipLaunchKernelGGL(k_pcg_update, dim3(G), dim3(kBlock), 0, s, n, rpb, h->w.p, h->v.p, h->d.p,
                     h->u.p, h->q.p, h->r.p, h->partials.p, h->counter.p, h->sc.p);
  AMG_LAUNCH_CHECK();
}
}  // namespace

void destroy_graph(amg_hierarchy *h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
}

int pcg_solve(amg_hierarchy *h, const double *b, double *x, double rtol, int maxit, int *iters,
              double *relres) {
  hipStream_t s = h->stream;
  const Level &L0 = h->L[0];
  const int n = L0.A.n, G = dot_blocks(n), rpb = rows_per_block(n, G);
  AMG_HIP(hipMemcpyAsync(h->u.p, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_zero<double>, grid_for(n), dim3(kBlock), 0, s, n, h->d.p);
  hipLaunchKernelGGL(k_zero<double>, grid_for(n), dim3(kBlock), 0, s, n, h->q.p);
  hipLaunchKernelGGL(k_pcg_init, dim3(G), dim3(kBlock), 0, s, n, rpb, L0.S.sptr.p, L0.S.col.p,
                     L0.S.val.p, b, h->u.p, h->r.p, h->partials.p, h->counter.p, h->sc.p, rtol);
  AMG_LAUNCH_CHECK();
  AMG_HIP(hipMemcpyAsync(h->sc_host, h->sc.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  Scalars st = *h->sc_host;
  if (st.status != 0) { *iters = 0; *relres = NAN; return st.status; }
  if (st.nr0 == 0.0) {
    AMG_HIP(hipMemcpyAsync(x, h->u.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipStreamSynchronize(s));
    *iters = 0;
    *relres = 0.0;
    return AMG_OK;
  }
  if (h->use_graph && !h->graph_exec) {
    AMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    enqueue_iteration(h);
    AMG_HIP(hipStreamEndCapture(s, &h->graph));
    AMG_HIP(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
  }
  int it = 0, status = AMG_OK;
  for (;;) {
    if (h->graph_exec) AMG_HIP(hipGraphLaunch(h->graph_exec, s));
    else enqueue_iteration(h);
    ++it;
    AMG_HIP(hipMemcpyAsync(h->sc_host, h->sc.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    st = *h->sc_host;
    if (st.status != 0) { status = st.status; break; }
    if (st.done) break;
    if (it >= maxit) { status = AMG_NOT_CONVERGED; break; }
  }
  AMG_HIP(hipMemcpyAsync(x, h->u.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  AMG_HIP(hipStreamSynchronize(s));
  *iters = it;
  *relres = sqrt(st.rr) / st.nr0;
  return status;
}

// ------------------------------------------------------- kernel timing
void time_kernel(amg_hierarchy *h, int kernel, int k, int reps, double *avg_ms, double *bytes) {
  hipStream_t s = h->stream;
  if (k < 0 || k >= static_cast<int>(h->L.size())) fail(AMG_ERR_INVALID, "level out of range");
  Level &L = h->L[k];
  const int n = L.A.n;
  const double nnz = static_cast<double>(L.A.nnz);
  const int G = dot_blocks(n), rpb = rows_per_block(n, G);
  auto launch = [&]() {
    switch (kernel) {
      case 0:
        if (k == 0) {
          hipLaunchKernelGGL(k_pcg_spmv_dots, dim3(G), dim3(kBlock), 0, s, n, rpb, L.S.sptr.p,
                             L.S.col.p, L.S.val.p, h->w.p, h->r.p, h->q.p, h->v.p, h->partials.p,
                             h->counter.p, h->sc.p);
        } else {
          hipLaunchKernelGGL(k_spmv<double>, grid_for(n), dim3(kBlock), 0, s, n, L.S.sptr.p,
                             L.S.col.p, L.S.val.p, L.x.p, L.t.p);
        }
        break;
      case 1:
        launch_sweep<double>(L, L.r.p, L.x.p, L.t.p, s);
        break;
      case 2:
        if (k + 1 >= static_cast<int>(h->L.size())) fail(AMG_ERR_INVALID, "no coarser level");
        hipLaunchKernelGGL(k_restrict<double>, grid_for(L.nc), dim3(kBlock), 0, s, L.nc, L.mptr.p,
                           L.mem.p, L.pval.p, L.S.sptr.p, L.S.col.p, L.S.val.p, L.r.p, L.x.p,
                           h->L[k + 1].r.p);
        break;
      case 3:
        if (k + 1 >= static_cast<int>(h->L.size())) fail(AMG_ERR_INVALID, "no coarser level");
        hipLaunchKernelGGL(k_prolong<double>, grid_for(n), dim3(kBlock), 0, s, n, L.agg.p, L.pval.p,
                           h->L[k + 1].x.p, L.t.p);
        break;
      case 4:
        if (k != 0) fail(AMG_ERR_INVALID, "the PCG update exists on level 0 only");
        hipLaunchKernelGGL(k_pcg_update, dim3(G), dim3(kBlock), 0, s, n, rpb, h->w.p, h->v.p, h->d.p,
                           h->u.p, h->q.p, h->r.p, h->partials.p, h->counter.p, h->sc.p);
        break;
      default:
        fail(AMG_ERR_INVALID, "unknown kernel id");
    }
    AMG_LAUNCH_CHECK();
  };
  // defined, finite inputs for the timed launches
  hipLaunchKernelGGL(k_zero<double>, grid_for(n), dim3(kBlock), 0, s, n, L.x.p);
  hipLaunchKernelGGL(k_zero<double>, grid_for(n), dim3(kBlock), 0, s, n, L.r.p);
  launch();
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  AMG_HIP(hipEventRecord(e0, s));
  for (int q = 0; q < reps; ++q) launch();
  AMG_HIP(hipEventRecord(e1, s));
  AMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = static_cast<double>(ms) / std::max(1, reps);
  const double bv = 8.0, nd = static_cast<double>(n), ncd = static_cast<double>(L.nc);
  switch (kernel) {
    case 0: *bytes = (bv + 4) * nnz + 2 * bv * nd + (k == 0 ? 2 * bv * nd : 0.0); break;
    case 1: *bytes = (bv + 4) * nnz + 3 * bv * nd; break;
    case 2: *bytes = (bv + 4) * nnz + 2 * bv * nd + (bv + 4) * nd + 4 * (ncd + 1) + bv * ncd; break;
    case 3: *bytes = 3 * bv * nd + 4 * nd + bv * ncd; break;
    default: *bytes = 10 * bv * nd; break;
  }
}

}  // namespace amg
