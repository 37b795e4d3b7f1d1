// Batched AMG-PCG: many independent s.p.d. systems of uneven size, each with
// several right-hand sides, solved together.
//
// Layout.  Every system gets its own hierarchy (the single-system setup,
// unchanged), then level k of all systems that reach level k is stacked into
// one block-diagonal matrix.  Systems are ordered by depth (deepest first),
// so at every level the active systems form a prefix, and the systems whose
// coarsest level is k come last ("terminal" rows).  Vectors are RHS-
// interleaved: entry (row i, right-hand side c) lives at i * NR + c, so one
// pass over a SELL matrix serves all NR right-hand sides.
//
// Each (system, right-hand side) pair is its own flexible CG (Alg. 1) with
// its own scalars and stopping test; a pair that has converged keeps its
// vectors frozen, so iteration counts are exact per pair.  Iterations are
// captured as one hipGraph (unrolled, masked) launched until every pair has
// converged.  Rows-per-wave of the smoothing and residual kernels (lanes per row
// = NR / columns-per-lane) are chosen per level by timing the candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <type_traits>
#include <vector>

#include "amg_internal.hpp"

namespace amg {
namespace {

// Rows per reduction tile of the level-0 PCG kernels.  The dot products
// fold per tile and then per system in tile order, so the tile size (and
// the SpMM's columns per thread) fix the rounding of every PCG scalar: they
// are constants, not tuned, so that a solve gives the same bits in every run
// (timing-dependent picks of 128-1024 rows and 1-4 columns measured within
// 2 % of these).
constexpr int kBTile = 256;
template <int NR>
constexpr int spmm_cols() { return NR % 2 == 0 ? 2 : 1; }

struct BScalars {
  double rho, c, a, rr, nr0, thr;
  int it, done, conv, status;
};

struct BLevel {
  int n = 0;        // rows of all systems active on this level
  int n_cont = 0;   // rows of the systems that continue below (a prefix)
  Level L;          // stacked matrix, l1 diagonals, transfer to the next level
  // systems whose coarsest level is this one (rows [n_cont, n))
  int nterm = 0;
  dvec<int> term_off, term_n;
  dvec<long long> term_inv;     // offset of each inverse in inv_pool
  dvec<double> inv_pool;        // column-major inverses of the coarsest matrices
  int cpl = 1;                  // tuned columns per lane (sweeps / residual)
  int cpl_corr = 1;             // tuned columns per lane of the corrected sweep
  int cpl_wide = 1;             // tuned columns per lane of the widening last sweep (level 0, binary32)
  int tune_best = 1;
  // RHS-interleaved work vectors
  dvec<double> r, x, t;
  dvec<float> rf, xf, tf;
};

inline dim3 grid_for(int64_t n, int block = kBlock) {
  return dim3(static_cast<unsigned>(std::max<int64_t>(1, (n + block - 1) / block)));
}

#define AMG_SKIP_IF_DONE() \
  if (skip && *skip) return

// Grids are capped at kMaxGrid workgroups.  The virtual blocks (kBlock
// threads each) are split into 8 contiguous eighths, one per XCD (workgroup
// b runs on XCD b % 8); the g workgroups of an XCD take its eighth in rounds
// of g consecutive blocks.  Each XCD thus sweeps one contiguous range of
// rows from start to end, and a row's neighbours a grid plane behind were
// read by the same XCD shortly before and are still in its L2.  (Striding
// the whole grid instead, every XCD jumped ahead by the grid's rows each
// round and fetched the planes around every jump again: 1.4-1.7x the
// algorithmic bytes on the 64-system fine level.)  An iteration queued
// after convergence costs little dispatch work.
#ifndef AMG_BATCH_MAX_GRID
#define AMG_BATCH_MAX_GRID 4096
#endif
constexpr int kMaxGrid = AMG_BATCH_MAX_GRID;

// Grid of a virtual-block kernel: the workgroups that fit on the device at
// once (the kernel's occupancy times the compute units, at most kMaxGrid),
// so that the rounds of vspan are walked by resident workgroups only and the
// rows in flight form one moving window per XCD.
template <class K>
int resident_workgroups(K kern) {
  struct Entry {
    const void *kern;
    int dev, grid;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  const void *key = reinterpret_cast<const void *>(kern);
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  for (const Entry &e : cache)
    if (e.kern == key && e.dev == dev) return e.grid;
  int cus = 0, occ = 0;
  AMG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  AMG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kBlock, 0));
  const int g = std::max(kXcd, std::min(kMaxGrid, occ * cus));
  cache.push_back(Entry{key, dev, g});
  return g;
}

template <class K>
dim3 rgrid(K kern, int64_t threads) {
  const int64_t nvb = std::max<int64_t>(1, (threads + kBlock - 1) / kBlock);
  return dim3(static_cast<unsigned>(std::min<int64_t>(nvb, resident_workgroups(kern))));
}


struct VSpan {
  int64_t b, e, step;
};

__device__ __forceinline__ VSpan vspan(int64_t threads) {
  const int64_t nvb = (threads + kBlock - 1) / kBlock;
  const int G = static_cast<int>(gridDim.x);
  const int x = static_cast<int>(blockIdx.x) % kXcd, j = static_cast<int>(blockIdx.x) / kXcd;
  const int gx = G / kXcd + (x < G % kXcd ? 1 : 0);   // workgroups on XCD x
  const int64_t chunk = (nvb + kXcd - 1) / kXcd;
  const int64_t b0 = static_cast<int64_t>(x) * chunk;
  const int64_t e0 = b0 + chunk < nvb ? b0 + chunk : nvb;
  return VSpan{b0 + j, e0, gx};
}

// ------------------------------------------------------------ stacking
__global__ void k_add_copy(int n, const int *__restrict__ src, int *__restrict__ dst, int add) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] + add;
}

__global__ void k_set_one(int *p, int v) { *p = v; }

// --------------------------------------------------------- SELL, NR columns
// CPL consecutive columns of one row of an RHS-interleaved vector, moved in
// 16-byte pieces when they fill them (rows are NR * sizeof(T) bytes apart and
// cb is a multiple of CPL, so such pieces are 16-byte aligned).
template <class T, int CPL>
__device__ __forceinline__ void ldcols(const T *__restrict__ p, T (&v)[CPL]) {
  constexpr int kVec = 16 / static_cast<int>(sizeof(T));
  if constexpr (CPL % kVec == 0) {
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
#pragma unroll
    for (int q = 0; q < CPL / kVec; ++q) {
      const V t = reinterpret_cast<const V *>(p)[q];
      __builtin_memcpy(&v[q * kVec], &t, 16);
    }
  } else {
#pragma unroll
    for (int j = 0; j < CPL; ++j) v[j] = p[j];
  }
}

template <class T, int CPL>
__device__ __forceinline__ void stcols(T *__restrict__ p, const T (&v)[CPL]) {
  constexpr int kVec = 16 / static_cast<int>(sizeof(T));
  if constexpr (CPL % kVec == 0) {
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
#pragma unroll
    for (int q = 0; q < CPL / kVec; ++q) {
      V t;
      __builtin_memcpy(&t, &v[q * kVec], 16);
      reinterpret_cast<V *>(p)[q] = t;
    }
  } else {
#pragma unroll
    for (int j = 0; j < CPL; ++j) p[j] = v[j];
  }
}

// y = x + p_c e[agg_c] at the kBS columns c[0 .. nv) of a batch: the P values
// and aggregate ids of the whole batch are loaded first, then its pieces of e.
template <class T, int NR, int CPL, int kBS>
__device__ __forceinline__ void correct(const int (&c)[kBS], int nv, const int *__restrict__ agg,
                                        const T *__restrict__ pval, const T *__restrict__ e, int cb,
                                        T (&xv)[kBS][CPL]) {
  T pc[kBS], ev[kBS][CPL];
  int g[kBS];
#pragma unroll
  for (int u = 0; u < kBS; ++u)
    if (u < nv) {
      pc[u] = pval[c[u]];
      g[u] = agg[c[u]];
    }
#pragma unroll
  for (int u = 0; u < kBS; ++u)
    if (u < nv) ldcols<T, CPL>(e + static_cast<int64_t>(g[u]) * NR + cb, ev[u]);
#pragma unroll
  for (int u = 0; u < kBS; ++u)
    if (u < nv)
#pragma unroll
      for (int j = 0; j < CPL; ++j) xv[u][j] = xv[u][j] + pc[u] * ev[u][j];
}

// Row `row`, columns cb .. cb+CPL-1: acc[j] = sum_k a_k x[col_k * NR + cb + j]
// folded in CSR order; l1 = sum_k |a_k|.  The iterate read at column c is
// x_c, or with a correction (e != nullptr) x_c + p_c e[agg_c] (the value the
// prolongation stores).  Slots are taken kBS at a time (columns, values,
// then the iterate pieces of the whole batch in flight before the fold;
// kBS keeps the batch's iterate pieces within 64 registers, so a 7-point
// row with pieces of up to 32 bytes is one batch: two dependent round trips
// per row).
template <class T, int NR, int CPL, bool kCorr = false>
__device__ __forceinline__ void brow(const int *__restrict__ sptr, const int *__restrict__ col,
                                     const T *__restrict__ val, const T *__restrict__ x, int row,
                                     int cb, T (&acc)[CPL], T &l1,
                                     const int *__restrict__ agg = nullptr,
                                     const T *__restrict__ pval = nullptr,
                                     const T *__restrict__ e = nullptr) {
  constexpr int kBytes = CPL * static_cast<int>(sizeof(T)) * (kCorr ? 2 : 1);
  constexpr int kBS = kBytes <= 32 ? 8 : (kBytes <= 64 ? 4 : (kBytes <= 128 ? 2 : 1));
  const int s = row >> 6, lane = row & 63;
  const int b = sptr[s], width = (sptr[s + 1] - b) >> 6;
#pragma unroll
  for (int j = 0; j < CPL; ++j) acc[j] = T(0);
  T m = T(0);
  int k = 0;
  if constexpr (kBS > 1) {
    for (; k + kBS <= width; k += kBS) {
      int c[kBS];
      T a[kBS], xv[kBS][CPL];
#pragma unroll
      for (int u = 0; u < kBS; ++u) {
        c[u] = col[b + (k + u) * 64 + lane];
        a[u] = val[b + (k + u) * 64 + lane];
      }
#pragma unroll
      for (int u = 0; u < kBS; ++u) ldcols<T, CPL>(x + static_cast<int64_t>(c[u]) * NR + cb, xv[u]);
      if constexpr (kCorr) correct<T, NR, CPL, kBS>(c, kBS, agg, pval, e, cb, xv);
#pragma unroll
      for (int u = 0; u < kBS; ++u) {
        m = m + fabs(a[u]);
#pragma unroll
        for (int j = 0; j < CPL; ++j) acc[j] = acc[j] + a[u] * xv[u][j];
      }
    }
    const int rem = width - k;   // 0 .. kBS-1, one predicated batch
    if (rem > 0) {
      int c[kBS];
      T a[kBS], xv[kBS][CPL];
#pragma unroll
      for (int u = 0; u < kBS; ++u)
        if (u < rem) {
          c[u] = col[b + (k + u) * 64 + lane];
          a[u] = val[b + (k + u) * 64 + lane];
        }
#pragma unroll
      for (int u = 0; u < kBS; ++u)
        if (u < rem) ldcols<T, CPL>(x + static_cast<int64_t>(c[u]) * NR + cb, xv[u]);
      if constexpr (kCorr) correct<T, NR, CPL, kBS>(c, rem, agg, pval, e, cb, xv);
#pragma unroll
      for (int u = 0; u < kBS; ++u)
        if (u < rem) {
          m = m + fabs(a[u]);
#pragma unroll
          for (int j = 0; j < CPL; ++j) acc[j] = acc[j] + a[u] * xv[u][j];
        }
      k = width;
    }
  }
  for (; k < width; ++k) {
    const int c = col[b + k * 64 + lane];
    const T a = val[b + k * 64 + lane];
    m = m + fabs(a);
    T xv[CPL];
    ldcols<T, CPL>(x + static_cast<int64_t>(c) * NR + cb, xv);
    if constexpr (kCorr) {
      const T pc = pval[c];
      T ev[CPL];
      ldcols<T, CPL>(e + static_cast<int64_t>(agg[c]) * NR + cb, ev);
#pragma unroll
      for (int j = 0; j < CPL; ++j) xv[j] = xv[j] + pc * ev[j];
    }
#pragma unroll
    for (int j = 0; j < CPL; ++j) acc[j] = acc[j] + a * xv[j];
  }
  l1 = m;
}

// Compact columns and value codes of a stacked level (the single-system SELL
// forms: 16-bit offsets from a per-slot-group base and one byte per slot
// naming an entry of the level's value table, both stored by quads of four
// slots per lane).  code == nullptr: the level has more than kDictMax
// distinct values and is read from col / val.
template <class T>
struct BCodes {
  const int *cbase, *qptr;
  const unsigned short *cdel;
  const unsigned char *code;
  const T *dict;
  int ndict;
};

// The value table in LDS (one copy per workgroup); called by every thread.
template <class T>
__device__ __forceinline__ void stage_bdict(const BCodes<T> &K, T *sd) {
  if (!K.code) return;   // uniform
  for (int i = threadIdx.x; i < K.ndict; i += blockDim.x) sd[i] = K.dict[i];
  __syncthreads();
}

// brow through the compact columns and codes: the same slots, values and
// fold order (slot order, padding slots included), so the same bits.
template <class T, int NR, int CPL, bool kCorr, int KB>
__device__ __forceinline__ void brow_coded(const BCodes<T> &K, const T *sd, int s, int b, int width,
                                           const T *__restrict__ x, int lane, int cb, T (&acc)[CPL],
                                           T &l1, const int *__restrict__ agg,
                                           const T *__restrict__ pval, const T *__restrict__ e) {
  const int64_t q = static_cast<int64_t>(K.qptr[s]) * 64 + lane;
  const unsigned long long *dq = reinterpret_cast<const unsigned long long *>(K.cdel) + q;
  const unsigned *cq = reinterpret_cast<const unsigned *>(K.code) + q;
  const int *bp = K.cbase + (b >> 6);
#pragma unroll
  for (int j = 0; j < CPL; ++j) acc[j] = T(0);
  T m = T(0);
  constexpr int QN = KB > 4 ? 2 : 1;   // quads per step: their loads, then all their gathers
  constexpr int SL = 4 * QN;
  for (int k0 = 0; k0 < width; k0 += SL) {
    int c[SL];
    T a[SL];
#pragma unroll
    for (int qn = 0; qn < QN; ++qn) {
      if (k0 + 4 * qn >= width) break;   // the slice's last quad
      const int64_t t = (k0 >> 2) + qn;
      const unsigned long long d = dq[t * 64];
      const unsigned w = cq[t * 64];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        c[4 * qn + j] = bp[k0 + 4 * qn + j] + static_cast<int>((d >> (16 * j)) & 0xffffu);   // cbase is padded
        a[4 * qn + j] = sd[(w >> (8 * j)) & 0xffu];
      }
    }
    const int nv = width - k0 < SL ? width - k0 : SL;
#pragma unroll
    for (int u0 = 0; u0 < SL; u0 += KB) {
      if (u0 >= nv) break;
      int cc[KB];
      T xv[KB][CPL];
      const int nb = nv - u0 < KB ? nv - u0 : KB;
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        cc[u] = c[u0 + u];
        if (u < nb) ldcols<T, CPL>(x + static_cast<int64_t>(cc[u]) * NR + cb, xv[u]);
      }
      if constexpr (kCorr) correct<T, NR, CPL, KB>(cc, nb, agg, pval, e, cb, xv);
#pragma unroll
      for (int u = 0; u < KB; ++u)
        if (u < nb) {
          m = m + fabs(a[u0 + u]);
#pragma unroll
          for (int jj = 0; jj < CPL; ++jj) acc[jj] = acc[jj] + a[u0 + u] * xv[u][jj];
        }
    }
  }
  l1 = m;
}

// Row `row` from the codes where its slice is compact and the level coded,
// else from col / val.
template <class T, int NR, int CPL, bool kCorr = false, bool kCO = false>
__device__ __forceinline__ void brow_k(const BCodes<T> &K, const T *sd, const int *__restrict__ sptr,
                                       const int *__restrict__ col, const T *__restrict__ val,
                                       const T *__restrict__ x, int row, int cb, T (&acc)[CPL], T &l1,
                                       const int *__restrict__ agg = nullptr,
                                       const T *__restrict__ pval = nullptr,
                                       const T *__restrict__ e = nullptr) {
  constexpr int kBytes = CPL * static_cast<int>(sizeof(T)) * (kCorr ? 2 : 1);
  // eight slots in flight for binary32 pieces of up to 32 bytes (two quads
  // per step); binary64 keeps four (the SpMM + dots measured slower with
  // eight: 1.79 vs 1.73 ms, its registers cost a wavefront)
  constexpr int KB = (kBytes <= 32 && sizeof(T) == 4) ? 8 : (kBytes <= 64 ? 4 : (kBytes <= 128 ? 2 : 1));
  if constexpr (kCO) {   // the level is coded and every slice compact: no plain path compiled
    const int s = row >> 6;
    const int b = sptr[s], width = (sptr[s + 1] - b) >> 6;
    brow_coded<T, NR, CPL, kCorr, KB>(K, sd, s, b, width, x, row & 63, cb, acc, l1, agg, pval, e);
  } else {
    if (K.code) {
      const int s = row >> 6;
      const int b = sptr[s], width = (sptr[s + 1] - b) >> 6;
      if (width > 0 && K.cbase[b >> 6] >= 0) {
        brow_coded<T, NR, CPL, kCorr, KB>(K, sd, s, b, width, x, row & 63, cb, acc, l1, agg, pval, e);
        return;
      }
    }
    brow<T, NR, CPL, kCorr>(sptr, col, val, x, row, cb, acc, l1, agg, pval, e);
  }
}

// xn = x + dinv (rhs - A x) on rows [0, n).  TO = double with T = float
// writes the binary32 result widened (exactly) to binary64: the last sweep
// of a binary32 cycle then delivers the binary64 output itself.
template <class T, int NR, int CPL, class TO = T, bool kCO = false>
__global__ void __launch_bounds__(kBlock) k_bsweep(const int *skip, int n,
                                                   const int *__restrict__ sptr,
                                                   const int *__restrict__ col,
                                                   const T *__restrict__ val,
                                                   const T *__restrict__ rhs,
                                                   const T *__restrict__ x, TO *__restrict__ xn,
                                                   BCodes<T> K) {
  AMG_SKIP_IF_DONE();
  __shared__ T sd[kDictMax];
  stage_bdict(K, sd);
  constexpr int LPR = NR / CPL;
  const VSpan sp = vspan(static_cast<int64_t>(n) * LPR);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
  const int64_t gid = vb * kBlock + threadIdx.x;
  const int row = static_cast<int>(gid / LPR), cb = static_cast<int>(gid % LPR) * CPL;
  if (row >= n) continue;
  T acc[CPL], l1;
  brow_k<T, NR, CPL, false, kCO>(K, sd, sptr, col, val, x, row, cb, acc, l1);
  const T di = T(1) / l1;
  const int64_t o = static_cast<int64_t>(row) * NR + cb;
  T xo[CPL], bo[CPL];
  TO out[CPL];
  ldcols<T, CPL>(x + o, xo);
  ldcols<T, CPL>(rhs + o, bo);
#pragma unroll
  for (int j = 0; j < CPL; ++j) out[j] = static_cast<TO>(xo[j] + di * (bo[j] - acc[j]));
  stcols<TO, CPL>(xn + o, out);
  }
}

// First post-smoothing sweep with the coarse correction folded in: the
// iterate read at column c is y_c = x_c + p_c e[agg_c] (the value k_bprolong
// stores), xn = y + dinv (rhs - A y); y is never written.  Rows [0, n) all
// continue to the coarser level.
template <class T, int NR, int CPL, bool kCO = false>
__global__ void __launch_bounds__(kBlock) k_bsweep_corr(const int *skip, int n,
                                                        const int *__restrict__ sptr,
                                                        const int *__restrict__ col,
                                                        const T *__restrict__ val,
                                                        const T *__restrict__ rhs,
                                                        const T *__restrict__ x,
                                                        const int *__restrict__ agg,
                                                        const T *__restrict__ pval,
                                                        const T *__restrict__ e, T *__restrict__ xn,
                                                        BCodes<T> K) {
  AMG_SKIP_IF_DONE();
  __shared__ T sd[kDictMax];
  stage_bdict(K, sd);
  constexpr int LPR = NR / CPL;
  const VSpan sp = vspan(static_cast<int64_t>(n) * LPR);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
  const int64_t gid = vb * kBlock + threadIdx.x;
  const int row = static_cast<int>(gid / LPR), cb = static_cast<int>(gid % LPR) * CPL;
  if (row >= n) continue;
  T acc[CPL], m;
  brow_k<T, NR, CPL, true, kCO>(K, sd, sptr, col, val, x, row, cb, acc, m, agg, pval, e);
  const T di = T(1) / m;
  const T pr = pval[row];
  const int64_t o = static_cast<int64_t>(row) * NR + cb;
  T xo[CPL], eo[CPL], bo[CPL], out[CPL];
  ldcols<T, CPL>(x + o, xo);
  ldcols<T, CPL>(e + static_cast<int64_t>(agg[row]) * NR + cb, eo);
  ldcols<T, CPL>(rhs + o, bo);
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const T y = xo[j] + pr * eo[j];
    out[j] = y + di * (bo[j] - acc[j]);
  }
  stcols<T, CPL>(xn + o, out);
  }
}

// t = p (rhs - A x) on rows [0, n)
template <class T, int NR, int CPL, bool kCO = false>
__global__ void __launch_bounds__(kBlock) k_bresid(const int *skip, int n,
                                                   const int *__restrict__ sptr,
                                                   const int *__restrict__ col,
                                                   const T *__restrict__ val,
                                                   const T *__restrict__ pval,
                                                   const T *__restrict__ rhs,
                                                   const T *__restrict__ x, T *__restrict__ t,
                                                   BCodes<T> K) {
  AMG_SKIP_IF_DONE();
  __shared__ T sd[kDictMax];
  stage_bdict(K, sd);
  constexpr int LPR = NR / CPL;
  const VSpan sp = vspan(static_cast<int64_t>(n) * LPR);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
  const int64_t gid = vb * kBlock + threadIdx.x;
  const int row = static_cast<int>(gid / LPR), cb = static_cast<int>(gid % LPR) * CPL;
  if (row >= n) continue;
  T acc[CPL], l1;
  brow_k<T, NR, CPL, false, kCO>(K, sd, sptr, col, val, x, row, cb, acc, l1);
  const T p = pval[row];
  const int64_t o = static_cast<int64_t>(row) * NR + cb;
  T bo[CPL], out[CPL];
  ldcols<T, CPL>(rhs + o, bo);
#pragma unroll
  for (int j = 0; j < CPL; ++j) out[j] = p * (bo[j] - acc[j]);
  stcols<T, CPL>(t + o, out);
  }
}

// x = dinv * rhs on rows [0, n)
template <class T, int NR>
__global__ void __launch_bounds__(kBlock) k_bsweep_first(const int *skip, int n,
                                                         const T *__restrict__ dinv,
                                                         const T *__restrict__ rhs,
                                                         T *__restrict__ x) {
  AMG_SKIP_IF_DONE();
  const int64_t m = static_cast<int64_t>(n) * NR;
  const VSpan sp = vspan(m);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
    const int64_t e = vb * kBlock + threadIdx.x;
    if (e < m) x[e] = dinv[e / NR] * rhs[e];
  }
}

// rc[I] = sum over members (ascending) of t; xc[I] = dinv_c[I] rc[I] when
// asked.  A thread takes ACPL columns of one aggregate; up to 8 member ids
// and their rows' pieces are in flight before the fold.
template <int NR>
constexpr int agg_cols() { return NR < 4 ? NR : 4; }

template <class T, int NR>
__global__ void __launch_bounds__(kBlock) k_bagg(const int *skip, int nc,
                                                 const int *__restrict__ mptr,
                                                 const int *__restrict__ mem,
                                                 const T *__restrict__ t, T *__restrict__ rc,
                                                 const T *__restrict__ dinvc, T *__restrict__ xc) {
  AMG_SKIP_IF_DONE();
  constexpr int ACPL = agg_cols<NR>(), LPA = NR / ACPL;
  const int64_t m = static_cast<int64_t>(nc) * LPA;
  const VSpan sp = vspan(m);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
    const int64_t e = vb * kBlock + threadIdx.x;
    if (e >= m) continue;
    const int I = static_cast<int>(e / LPA), cb = static_cast<int>(e % LPA) * ACPL;
    const int q0 = mptr[I], q1 = mptr[I + 1];
    T acc[ACPL];
#pragma unroll
    for (int j = 0; j < ACPL; ++j) acc[j] = T(0);
    int q = q0;
    for (; q < q1; q += 8) {
      const int nm = q1 - q < 8 ? q1 - q : 8;
      int mm[8];
      T v[8][ACPL];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < nm) mm[u] = mem[q + u];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < nm) ldcols<T, ACPL>(t + static_cast<int64_t>(mm[u]) * NR + cb, v[u]);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < nm)
#pragma unroll
          for (int j = 0; j < ACPL; ++j) acc[j] = acc[j] + v[u][j];
    }
    const int64_t o = static_cast<int64_t>(I) * NR + cb;
    stcols<T, ACPL>(rc + o, acc);
    if (xc) {
      const T di = dinvc[I];
      T xo[ACPL];
#pragma unroll
      for (int j = 0; j < ACPL; ++j) xo[j] = di * acc[j];
      stcols<T, ACPL>(xc + o, xo);
    }
  }
}

// x += p e[agg] on rows [0, n)
template <class T, int NR>
__global__ void __launch_bounds__(kBlock) k_bprolong(const int *skip, int n,
                                                     const int *__restrict__ agg,
                                                     const T *__restrict__ pval,
                                                     const T *__restrict__ e, T *__restrict__ x) {
  AMG_SKIP_IF_DONE();
  const int64_t m = static_cast<int64_t>(n) * NR;
  const VSpan sp = vspan(m);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
    const int64_t q = vb * kBlock + threadIdx.x;
    if (q >= m) continue;
    const int i = static_cast<int>(q / NR), c = static_cast<int>(q % NR);
    x[q] = x[q] + pval[i] * e[static_cast<int64_t>(agg[i]) * NR + c];
  }
}

// Terminal systems: z = A_c^-1 r for all NR right-hand sides at once, one
// workgroup per system: the dense n x n inverse (column-major) times the
// n x NR block of right-hand sides, the one dense product of the method,
// on the FP64 matrix cores.  Each wavefront computes 16-row tiles of z with
// v_mfma_f64_16x16x4f64 over k in steps of 4: lane l supplies
// A[i0 + l % 16][k0 + l / 16] and R[k0 + l / 16][l % 16] and receives
// z[i0 + 4 q + l / 16][l % 16] in accumulator q (rows past n and columns
// past NR are zero-padded and not stored).  The sums round in the matrix
// core's order rather than the sequential fold's (relative difference of
// the order of the binary64 unit).
typedef double v4d __attribute__((ext_vector_type(4)));

template <class T, int NR>
__global__ void __launch_bounds__(kBlock) k_bcoarse(const int *skip, const int *__restrict__ toff,
                                                    const int *__restrict__ tn,
                                                    const long long *__restrict__ tinv,
                                                    const double *__restrict__ pool,
                                                    const T *__restrict__ rhs, T *__restrict__ out) {
  AMG_SKIP_IF_DONE();
  const int sys = blockIdx.x;
  const int off = toff[sys], n = tn[sys];
  const double *Ai = pool + tinv[sys];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int li = lane % 16, lk = lane / 16;
  const int ntile = (n + 15) / 16;
  for (int tile = wave; tile < ntile; tile += kBlock / kWave) {
    const int i = tile * 16 + li;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += 4) {
      const int k = k0 + lk;
      const double a = (i < n && k < n) ? Ai[static_cast<int64_t>(k) * n + i] : 0.0;
      const double b = (k < n && li < NR) ? static_cast<double>(rhs[static_cast<int64_t>(off + k) * NR + li]) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = tile * 16 + 4 * q + lk;
      if (row < n && li < NR) out[static_cast<int64_t>(off + row) * NR + li] = static_cast<T>(acc[q]);
    }
  }
}

// Entry of the binary32 cycle: rf = (float) r on all m entries and, on the
// first m1 entries (rows that smooth), the first iterate x = dinv_f * rf.
template <int NR>
__global__ void k_bd2f_first(int64_t m, int64_t m1, const double *__restrict__ r,
                             const float *__restrict__ dinv, float *__restrict__ rf,
                             float *__restrict__ x, const int *skip) {
  AMG_SKIP_IF_DONE();
  const VSpan sp = vspan(m);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
    const int64_t e = vb * kBlock + threadIdx.x;
    if (e >= m) continue;
    const float b = static_cast<float>(r[e]);
    rf[e] = b;
    if (x && e < m1) x[e] = dinv[e / NR] * b;
  }
}

__global__ void k_bf2d(int64_t m, const float *__restrict__ a, double *__restrict__ b,
                       const int *skip) {
  AMG_SKIP_IF_DONE();
  const VSpan sp = vspan(m);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
    const int64_t e = vb * kBlock + threadIdx.x;
    if (e < m) b[e] = static_cast<double>(a[e]);
  }
}

template <class T>
__global__ void k_bzero(int64_t m, T *x) {
  const VSpan sp = vspan(m);
  for (int64_t vb = sp.b; vb < sp.e; vb += sp.step) {
    const int64_t e = vb * kBlock + threadIdx.x;
    if (e < m) x[e] = T(0);
  }
}

// ------------------------------------------------------- level-0 PCG kernels
// A tile is <= kBTile rows of one system.  In the SpMV kernels a thread
// handles PC = min(4, NR) consecutive columns of one row at a time (lanes
// per row NR / PC); thread (rsub, cg) takes rows r0 + rsub, r0 + rsub +
// kBlock / (NR / PC), ...  The partial of column c folds the threads with that
// column in increasing rsub.
template <int NR>
constexpr int pcg_cols() { return NR < 4 ? NR : 4; }

template <int NR>
__device__ __forceinline__ double tile_column_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < NR)
    for (int g = 0; g < kBlock / NR; ++g) s = s + red[g * NR + threadIdx.x];
  __syncthreads();
  return s;
}

// Column sums of per-thread values v[j] (column cg * PC + j); the result for
// column c is returned to thread c < NR.
template <int NR, int PC>
__device__ __forceinline__ double tile_column_sum_v(const double (&v)[PC], double *red) {
  constexpr int LPR = NR / PC;
#pragma unroll
  for (int j = 0; j < PC; ++j) red[threadIdx.x * PC + j] = v[j];
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < NR) {
    const int cg = threadIdx.x / PC, j = threadIdx.x % PC;
    for (int g = 0; g < kBlock / LPR; ++g) s = s + red[(g * LPR + cg) * PC + j];
  }
  __syncthreads();
  return s;
}

// The binary32 cycle's entry, written by the kernels that produce r (the
// PCG init and update) instead of a pass of its own: rf = (float) r and, on
// the first m1 entries (rows that smooth), the first iterate xf = dinvf rf.
// rf == nullptr: not wanted (binary64 cycle, or no preconditioner).
struct BFirst {
  const float *dinvf;
  float *rf, *xf;
  int64_t m1;
  __device__ __forceinline__ void put(int64_t o, int row, double r) const {
    if (!rf) return;
    const float b = static_cast<float>(r);
    rf[o] = b;
    if (xf && o < m1) xf[o] = dinvf[row] * b;
  }
};

template <int NR>
__global__ void __launch_bounds__(kBlock) k_bpcg_init(const int *__restrict__ trow0,
                                                      const int *__restrict__ trow1,
                                                      const int *__restrict__ sptr,
                                                      const int *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ b,
                                                      const double *__restrict__ u,
                                                      double *__restrict__ r,
                                                      double *__restrict__ part,
                                                      BCodes<double> K, BFirst F) {
  constexpr int PC = pcg_cols<NR>(), LPR = NR / PC;
  __shared__ double red[kBlock * PC];
  __shared__ double sd[kDictMax];
  stage_bdict(K, sd);
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int cb = (threadIdx.x % LPR) * PC;
  double rr[PC];
#pragma unroll
  for (int j = 0; j < PC; ++j) rr[j] = 0.0;
  for (int row = trow0[tile] + threadIdx.x / LPR; row < trow1[tile]; row += kBlock / LPR) {
    double acc[PC], l1, bo[PC], ro[PC];
    brow_k<double, NR, PC>(K, sd, sptr, col, val, u, row, cb, acc, l1);
    const int64_t o = static_cast<int64_t>(row) * NR + cb;
    ldcols<double, PC>(b + o, bo);
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      ro[j] = bo[j] - acc[j];
      rr[j] = rr[j] + ro[j] * ro[j];
      F.put(o + j, row, ro[j]);
    }
    stcols<double, PC>(r + o, ro);
  }
  const double t = tile_column_sum_v<NR, PC>(rr, red);
  if (threadIdx.x < NR) part[(static_cast<int64_t>(tile) * NR + threadIdx.x) * 3] = t;
}

// PC columns per thread (tuned: fewer columns hold fewer gathered values in
// registers and let more waves run).
template <int NR, int PC, bool kCO = false>
__global__ void __launch_bounds__(kBlock) k_bpcg_spmm_dots(
    const int *skip, int ntiles, const int *__restrict__ trow0, const int *__restrict__ trow1,
    const int *__restrict__ sptr, const int *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ w, const double *__restrict__ r, const double *__restrict__ q,
    double *__restrict__ v, double *__restrict__ part, BCodes<double> K) {
  AMG_SKIP_IF_DONE();
  __shared__ double sd[kDictMax];
  stage_bdict(K, sd);
  constexpr int LPR = NR / PC;
  __shared__ double red[kBlock * PC];
  const int cb = (threadIdx.x % LPR) * PC;
  const VSpan sp = vspan(static_cast<int64_t>(ntiles) * kBlock);
  for (int64_t vt = sp.b; vt < sp.e; vt += sp.step) {
  const int tile = static_cast<int>(vt);
  double al[PC], be[PC], ga[PC];
#pragma unroll
  for (int j = 0; j < PC; ++j) al[j] = be[j] = ga[j] = 0.0;
  for (int row = trow0[tile] + threadIdx.x / LPR; row < trow1[tile]; row += kBlock / LPR) {
    double acc[PC], l1, wo[PC], ro[PC], qo[PC];
    brow_k<double, NR, PC, false, kCO>(K, sd, sptr, col, val, w, row, cb, acc, l1);
    const int64_t o = static_cast<int64_t>(row) * NR + cb;
    stcols<double, PC>(v + o, acc);
    ldcols<double, PC>(w + o, wo);
    ldcols<double, PC>(r + o, ro);
    ldcols<double, PC>(q + o, qo);
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      al[j] = al[j] + wo[j] * ro[j];
      be[j] = be[j] + wo[j] * acc[j];
      ga[j] = ga[j] + wo[j] * qo[j];
    }
  }
  const double sa = tile_column_sum_v<NR, PC>(al, red);
  const double sb = tile_column_sum_v<NR, PC>(be, red);
  const double sg = tile_column_sum_v<NR, PC>(ga, red);
  if (threadIdx.x < NR) {
    const int64_t o = (static_cast<int64_t>(tile) * NR + threadIdx.x) * 3;
    part[o] = sa;
    part[o + 1] = sb;
    part[o + 2] = sg;
  }
  }
}

// Fold the tiles of system `blockIdx.x` per column: thread (g, c) folds tiles
// g, g + G, ... in order (loads issued four tiles at a time); then the G
// group sums are folded in order.  One workgroup of kBFinish threads.
constexpr int kBFinish = 1024;

template <int NR, int NQ>
__device__ __forceinline__ void system_fold(const int *tile_ptr, const double *part, double *red,
                                            double (&out)[NQ]) {
  constexpr int G = kBFinish / NR;
  const int sys = blockIdx.x, c = threadIdx.x % NR, g = threadIdx.x / NR;
  double acc[NQ];
#pragma unroll
  for (int o = 0; o < NQ; ++o) acc[o] = 0.0;
  const int t1 = tile_ptr[sys + 1];
  int t = tile_ptr[sys] + g;
  for (; t + 3 * G < t1; t += 4 * G) {
    double v[4][NQ];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int o = 0; o < NQ; ++o) v[u][o] = part[(static_cast<int64_t>(t + u * G) * NR + c) * 3 + o];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int o = 0; o < NQ; ++o) acc[o] = acc[o] + v[u][o];
  }
  for (; t < t1; t += G)
#pragma unroll
    for (int o = 0; o < NQ; ++o) acc[o] = acc[o] + part[(static_cast<int64_t>(t) * NR + c) * 3 + o];
#pragma unroll
  for (int o = 0; o < NQ; ++o) {
    red[threadIdx.x] = acc[o];
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x < NR)
      for (int q = 0; q < G; ++q) s = s + red[q * NR + threadIdx.x];
    out[o] = s;
    __syncthreads();
  }
}

template <int NR>
__global__ void __launch_bounds__(kBFinish) k_bpcg_init_finish(const int *tile_ptr,
                                                             const double *part, BScalars *sc,
                                                             double rtol, int *active) {
  __shared__ double red[kBFinish];
  double t[1];
  system_fold<NR, 1>(tile_ptr, part, red, t);
  if (threadIdx.x < NR) {
    BScalars &S = sc[blockIdx.x * NR + threadIdx.x];
    const double nr0 = sqrt(t[0]);
    S.nr0 = nr0;
    S.rr = t[0];
    S.thr = rtol * nr0;
    S.rho = 1.0;
    S.c = 0.0;
    S.a = 0.0;
    S.it = 0;
    S.conv = (nr0 == 0.0) ? 1 : 0;
    S.status = isfinite(nr0) ? 0 : AMG_ERR_NONFINITE;
    S.done = (nr0 == 0.0 || !isfinite(nr0)) ? 1 : 0;
    if (!S.done) atomicAdd(active, 1);
  }
}

template <int NR>
__global__ void __launch_bounds__(kBFinish) k_bpcg_dots_finish(const int *skip, const int *tile_ptr,
                                                             const double *part, BScalars *sc) {
  AMG_SKIP_IF_DONE();
  __shared__ double red[kBFinish];
  double t[3];
  system_fold<NR, 3>(tile_ptr, part, red, t);
  if (threadIdx.x < NR) {
    BScalars &S = sc[blockIdx.x * NR + threadIdx.x];
    if (S.done) return;
    const double A = t[0], B = t[1], G = t[2];
    const double rho_prev = S.rho;
    const double rho = B - (G * G) / rho_prev;
    S.it = S.it + 1;
    if (!isfinite(rho) || !isfinite(A)) {
      S.status = AMG_ERR_NONFINITE;
      S.done = 1;
      return;
    }
    if (!(rho > 0.0)) {
      S.status = AMG_ERR_NOT_SPD;
      S.done = 1;
      return;
    }
    S.c = G / rho_prev;
    S.a = A / rho;
    S.rho = rho;
  }
}

// d = w - c d; u += a d; q = v - c q; r -= a q for live pairs; partial ||r||^2.
template <int NR>
__global__ void __launch_bounds__(kBlock) k_bpcg_update(
    const int *skip, int ntiles, const int *__restrict__ trow0, const int *__restrict__ trow1,
    const int *__restrict__ tsys, const double *__restrict__ w, const double *__restrict__ v,
    double *__restrict__ d, double *__restrict__ u, double *__restrict__ q, double *__restrict__ r,
    const BScalars *__restrict__ sc, double *__restrict__ part, BFirst F) {
  AMG_SKIP_IF_DONE();
  __shared__ double red[kBlock];
  const int c = threadIdx.x % NR;
  const VSpan sp = vspan(static_cast<int64_t>(ntiles) * kBlock);
  for (int64_t vt = sp.b; vt < sp.e; vt += sp.step) {
  const int tile = static_cast<int>(vt);
  const BScalars &S = sc[tsys[tile] * NR + c];
  const bool live = !S.done;
  const double cc = S.c, a = S.a;
  double rr = 0.0;
  if (live) {
    // w, v, d, u, q are not read again before the next update: non-temporal
    // accesses keep r (read by the next V-cycle) and the matrix in cache
    for (int row = trow0[tile] + threadIdx.x / NR; row < trow1[tile]; row += kBlock / NR) {
      const int64_t o = static_cast<int64_t>(row) * NR + c;
      const double di = ld_stream(w + o) - cc * ld_stream(d + o);
      __builtin_nontemporal_store(di, d + o);
      __builtin_nontemporal_store(ld_stream(u + o) + a * di, u + o);
      const double qi = ld_stream(v + o) - cc * ld_stream(q + o);
      __builtin_nontemporal_store(qi, q + o);
      const double ri = r[o] - a * qi;
      r[o] = ri;
      rr = rr + ri * ri;
      F.put(o, row, ri);   // frozen pairs keep their last entry values: their columns are unused
    }
  }
  rr = tile_column_sum<NR>(rr, red);
  if (threadIdx.x < NR) part[(static_cast<int64_t>(tile) * NR + c) * 3] = rr;
  }
}

template <int NR>
__global__ void __launch_bounds__(kBFinish) k_bpcg_norm_finish(const int *skip, const int *tile_ptr,
                                                             const double *part, BScalars *sc,
                                                             int maxit, int *active) {
  AMG_SKIP_IF_DONE();
  __shared__ double red[kBFinish];
  double t[1];
  system_fold<NR, 1>(tile_ptr, part, red, t);
  if (threadIdx.x < NR) {
    BScalars &S = sc[blockIdx.x * NR + threadIdx.x];
    if (S.done) return;
    const double nr = sqrt(t[0]);
    S.rr = t[0];
    if (nr <= S.thr) {
      S.conv = 1;
      S.done = 1;
    } else if (!isfinite(nr)) {
      S.status = AMG_ERR_NONFINITE;
      S.done = 1;
    } else if (S.it >= maxit) {
      S.done = 1;
    }
    if (!S.done) atomicAdd(active, 1);
  }
}

// all_done = (no live pair); the counter restarts; snapshot for the host.
__global__ void k_ball_done(int *active, int *all_done, int *host_flag) {
  const int live = *active;
  *all_done = (live == 0) ? 1 : 0;
  *active = 0;
  *host_flag = (live == 0) ? 1 : 0;
}

}  // namespace
}  // namespace amg

// ===================================================================
struct amg_batch {
  amg_params p{};
  hipStream_t stream = nullptr;
  bool own_stream = false;     // stream from acquire_private_stream (on stream_dev)
  int stream_dev = 0;
  int nsys = 0;
  std::vector<int> order;              // internal position -> user system id
  std::vector<int> pos_of;             // user system id -> internal position
  std::vector<int> nl;                 // levels per internal position
  std::vector<int64_t> n0;             // level-0 rows per user system
  std::vector<int64_t> user_off, int_off;   // level-0 row offsets (user order / internal order)
  std::vector<amg::BLevel> B;
  std::vector<int64_t> roff0;          // level-0 row offsets per internal position
  int ntiles = 0, tile_rows = 0, max_tiles = 0;
  int spmm_cols = 1;                   // columns per thread of the level-0 SpMM + dots
  amg::dvec<int> trow0, trow1, tsys, tile_ptr;
  // per-nrhs state
  int nr = 0;
  amg::dvec<double> bint, u, r, w, v, d, q, partials;
  amg::dvec<amg::BScalars> sc;
  amg::dvec<int> active, all_done;
  int *host_flag = nullptr, *host_flag_dev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_reps = 0, graph_maxit = 0;
  double setup_ms = 0.0, tune_ms = 0.0;
  int64_t nnz0 = 0;
};

namespace amg {
namespace {

template <class T> T *bv_r(BLevel &L);
template <> double *bv_r<double>(BLevel &L) { return L.r.p; }
template <> float *bv_r<float>(BLevel &L) { return L.rf.p; }
template <class T> T *bv_x(BLevel &L);
template <> double *bv_x<double>(BLevel &L) { return L.x.p; }
template <> float *bv_x<float>(BLevel &L) { return L.xf.p; }
template <class T> T *bv_t(BLevel &L);
template <> double *bv_t<double>(BLevel &L) { return L.t.p; }
template <> float *bv_t<float>(BLevel &L) { return L.tf.p; }
template <class T> const T *bvals(const Level &L);
template <> const double *bvals<double>(const Level &L) { return L.S.val.p; }
template <> const float *bvals<float>(const Level &L) { return L.S.valf.p; }
template <class T> const T *bdinv(const Level &L);
template <> const double *bdinv<double>(const Level &L) { return L.dinv.p; }
template <> const float *bdinv<float>(const Level &L) { return L.dinvf.p; }
template <class T> const T *bpval(const Level &L);
template <> const double *bpval<double>(const Level &L) { return L.pval.p; }
template <> const float *bpval<float>(const Level &L) { return L.pvalf.p; }
template <class T> const T *bdict(const Sell &S);
template <> const double *bdict<double>(const Sell &S) { return S.dict.p; }
template <> const float *bdict<float>(const Sell &S) { return S.dictf.p; }
template <class T>
BCodes<T> bcodes(const Level &L) {
  const Sell &S = L.S;
  const bool coded = S.ndict > 0 && S.cdel.p && S.code.p;
  return BCodes<T>{S.cbase.p, S.qptr.p, S.cdel.p, coded ? S.code.p : nullptr, bdict<T>(S), S.ndict};
}

// Every slice compact and the values coded: the kernels without the plain path.
inline bool coded_only(const Level &L) {
  return L.S.ndict > 0 && L.S.nslots > 0 && L.S.groups_compact * kSlice == L.S.nslots;
}

template <class T, int NR, int CPL, class TO, bool kCO>
void launch_bsweep_as(const int *skip, BLevel &L, int n, const T *rhs, const T *x, TO *xn, hipStream_t s) {
  constexpr int LPR = NR / CPL;
  auto kern = k_bsweep<T, NR, CPL, TO, kCO>;
  hipLaunchKernelGGL(kern, rgrid(kern, static_cast<int64_t>(n) * LPR), dim3(kBlock), 0, s, skip, n,
                     L.L.S.sptr.p, L.L.S.col.p, bvals<T>(L.L), rhs, x, xn, bcodes<T>(L.L));
}

template <class T, int NR, int CPL>
void launch_bsweep(const int *skip, BLevel &L, int n, const T *rhs, const T *x, T *xn, hipStream_t s) {
  if (coded_only(L.L)) launch_bsweep_as<T, NR, CPL, T, true>(skip, L, n, rhs, x, xn, s);
  else launch_bsweep_as<T, NR, CPL, T, false>(skip, L, n, rhs, x, xn, s);
}

template <int NR, int CPL>
void launch_bsweep_widen(const int *skip, BLevel &L, int n, const float *rhs, const float *x,
                         double *xn, hipStream_t s) {
  if (coded_only(L.L)) launch_bsweep_as<float, NR, CPL, double, true>(skip, L, n, rhs, x, xn, s);
  else launch_bsweep_as<float, NR, CPL, double, false>(skip, L, n, rhs, x, xn, s);
}

template <class T, int NR, int CPL, bool kCO>
void launch_bresid_as(const int *skip, BLevel &L, int n, const T *rhs, const T *x, T *t, hipStream_t s) {
  constexpr int LPR = NR / CPL;
  auto kern = k_bresid<T, NR, CPL, kCO>;
  hipLaunchKernelGGL(kern, rgrid(kern, static_cast<int64_t>(n) * LPR), dim3(kBlock), 0, s, skip, n,
                     L.L.S.sptr.p, L.L.S.col.p, bvals<T>(L.L), bpval<T>(L.L), rhs, x, t, bcodes<T>(L.L));
}

template <class T, int NR, int CPL>
void launch_bresid(const int *skip, BLevel &L, int n, const T *rhs, const T *x, T *t, hipStream_t s) {
  if (coded_only(L.L)) launch_bresid_as<T, NR, CPL, true>(skip, L, n, rhs, x, t, s);
  else launch_bresid_as<T, NR, CPL, false>(skip, L, n, rhs, x, t, s);
}

template <class T, int NR, int CPL, bool kCO>
void launch_bsweep_corr_as(const int *skip, BLevel &L, int n, const T *rhs, const T *e, const T *x, T *xn,
                           hipStream_t s) {
  constexpr int LPR = NR / CPL;
  auto kern = k_bsweep_corr<T, NR, CPL, kCO>;
  hipLaunchKernelGGL(kern, rgrid(kern, static_cast<int64_t>(n) * LPR), dim3(kBlock), 0, s, skip, n,
                     L.L.S.sptr.p, L.L.S.col.p, bvals<T>(L.L), rhs, x, L.L.agg.p, bpval<T>(L.L), e, xn,
                     bcodes<T>(L.L));
}

template <class T, int NR, int CPL>
void launch_bsweep_corr(const int *skip, BLevel &L, int n, const T *rhs, const T *e, const T *x, T *xn,
                        hipStream_t s) {
  if (coded_only(L.L)) launch_bsweep_corr_as<T, NR, CPL, true>(skip, L, n, rhs, e, x, xn, s);
  else launch_bsweep_corr_as<T, NR, CPL, false>(skip, L, n, rhs, e, x, xn, s);
}

// Calls f(std::integral_constant<int, C>) with C = cpl when cpl divides NR
// and is one of 1, 2, 4, 8, 16; else with C = 1.
template <int NR, class F>
void with_cpl(int cpl, F &&f) {
  if constexpr (NR % 16 == 0) if (cpl == 16) return f(std::integral_constant<int, 16>{});
  if constexpr (NR % 8 == 0) if (cpl == 8) return f(std::integral_constant<int, 8>{});
  if constexpr (NR % 4 == 0) if (cpl == 4) return f(std::integral_constant<int, 4>{});
  if constexpr (NR % 2 == 0) if (cpl == 2) return f(std::integral_constant<int, 2>{});
  return f(std::integral_constant<int, 1>{});
}

template <class T, int NR>
void corr_sweep_any(const int *skip, BLevel &L, int n, const T *rhs, const T *e, const T *x, T *xn,
                    hipStream_t s) {
  with_cpl<NR>(L.cpl_corr, [&](auto C) { launch_bsweep_corr<T, NR, decltype(C)::value>(skip, L, n, rhs, e, x, xn, s); });
}

template <class T, int NR>
void sweep_any(const int *skip, BLevel &L, int n, const T *rhs, const T *x, T *xn, hipStream_t s) {
  with_cpl<NR>(L.cpl, [&](auto C) { launch_bsweep<T, NR, decltype(C)::value>(skip, L, n, rhs, x, xn, s); });
}

template <int NR>
void sweep_widen_any(const int *skip, BLevel &L, int n, const float *rhs, const float *x, double *xn,
                     hipStream_t s) {
  with_cpl<NR>(L.cpl_wide, [&](auto C) { launch_bsweep_widen<NR, decltype(C)::value>(skip, L, n, rhs, x, xn, s); });
}

template <class T, int NR>
void resid_any(const int *skip, BLevel &L, int n, const T *rhs, const T *x, T *t, hipStream_t s) {
  with_cpl<NR>(L.cpl, [&](auto C) { launch_bresid<T, NR, decltype(C)::value>(skip, L, n, rhs, x, t, s); });
}

// first iterate location of level k (nullptr: no smoothing on this level)
template <class T>
T *bfirst(amg_batch *bt, int k, T *out) {
  BLevel &L = bt->B[k];
  const amg_params &P = bt->p;
  if (L.n_cont == 0 || P.pre_sweeps == 0) return nullptr;
  const int swaps = (P.pre_sweeps - 1) + P.post_sweeps;
  return (swaps % 2 == 0) ? out : bv_t<T>(L);
}

// What the PCG kernels write for the binary32 cycle's entry (none otherwise).
template <int NR>
BFirst bfirst_out(amg_batch *bt) {
  if (!bt->p.precond || bt->p.precision != AMG_PREC_MIXED) return BFirst{nullptr, nullptr, nullptr, 0};
  BLevel &L = bt->B[0];
  return BFirst{L.L.dinvf.p, L.rf.p, bfirst<float>(bt, 0, L.xf.p), static_cast<int64_t>(L.n_cont) * NR};
}

// z64 (binary32 cycle, level 0 only): the last post-sweep writes its rows
// there, widened, instead of into `out`; returns whether it did.
template <class T, int NR>
bool bvcycle_level(amg_batch *bt, const int *skip, int k, const T *rhs, T *out, bool first_done,
                   double *z64 = nullptr) {
  hipStream_t s = bt->stream;
  BLevel &L = bt->B[k];
  const amg_params &P = bt->p;
  const int nc0 = L.n_cont;
  if (L.nterm > 0)
    hipLaunchKernelGGL((k_bcoarse<T, NR>), dim3(L.nterm), dim3(kBlock), 0, s, skip, L.term_off.p,
                       L.term_n.p, L.term_inv.p, L.inv_pool.p, rhs, out);
  if (nc0 == 0) return false;
  const int swaps = (P.pre_sweeps > 0 ? P.pre_sweeps - 1 : 0) + P.post_sweeps;
  T *A = (swaps % 2 == 0) ? out : bv_t<T>(L);
  T *Bf = (A == out) ? bv_t<T>(L) : out;
  if (P.pre_sweeps == 0) {
    hipLaunchKernelGGL(k_bzero<T>, rgrid(k_bzero<T>, static_cast<int64_t>(nc0) * NR), dim3(kBlock), 0, s,
                       static_cast<int64_t>(nc0) * NR, A);
  } else {
    if (!first_done)
      hipLaunchKernelGGL((k_bsweep_first<T, NR>), rgrid((k_bsweep_first<T, NR>), static_cast<int64_t>(nc0) * NR), dim3(kBlock),
                         0, s, skip, nc0, bdinv<T>(L.L), rhs, A);
    for (int qq = 1; qq < P.pre_sweeps; ++qq) { sweep_any<T, NR>(skip, L, nc0, rhs, A, Bf, s); std::swap(A, Bf); }
  }
  resid_any<T, NR>(skip, L, nc0, rhs, A, Bf, s);
  BLevel &C = bt->B[k + 1];
  T *xc = bfirst<T>(bt, k + 1, bv_x<T>(C));
  hipLaunchKernelGGL((k_bagg<T, NR>), rgrid((k_bagg<T, NR>), static_cast<int64_t>(C.n) * (NR / agg_cols<NR>())), dim3(kBlock), 0, s, skip,
                     C.n, L.L.mptr.p, L.L.mem.p, Bf, bv_r<T>(C), bdinv<T>(C.L), xc);
  (void)bvcycle_level<T, NR>(bt, skip, k + 1, bv_r<T>(C), bv_x<T>(C), xc != nullptr);
  if (P.post_sweeps == 0) {
    hipLaunchKernelGGL((k_bprolong<T, NR>), rgrid((k_bprolong<T, NR>), static_cast<int64_t>(nc0) * NR), dim3(kBlock), 0, s,
                       skip, nc0, L.L.agg.p, bpval<T>(L.L), bv_x<T>(C), A);
    return false;
  }
  corr_sweep_any<T, NR>(skip, L, nc0, rhs, bv_x<T>(C), A, Bf, s);
  std::swap(A, Bf);
  const bool widen = std::is_same<T, float>::value && z64 && P.post_sweeps >= 2;
  for (int qq = 1; qq < P.post_sweeps; ++qq) {
    if (widen && qq == P.post_sweeps - 1) {
      if constexpr (std::is_same<T, float>::value) sweep_widen_any<NR>(skip, L, nc0, rhs, A, z64, s);
      return true;
    }
    sweep_any<T, NR>(skip, L, nc0, rhs, A, Bf, s);
    std::swap(A, Bf);
  }
  return false;
}

template <int NR>
void bvcycle(amg_batch *bt, const int *skip, const double *r, double *z, bool entry_done = false) {
  hipStream_t s = bt->stream;
  const int64_t m = static_cast<int64_t>(bt->B[0].n) * NR;
  if (!bt->p.precond) {
    AMG_HIP(hipMemcpyAsync(z, r, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    return;
  }
  if (bt->p.precision == AMG_PREC_MIXED) {
    BLevel &L = bt->B[0];
    float *x1 = bfirst<float>(bt, 0, L.xf.p);
    if (!entry_done)   // else the kernel that produced r wrote rf and x1 (bfirst_out)
      hipLaunchKernelGGL((k_bd2f_first<NR>), rgrid((k_bd2f_first<NR>), m), dim3(kBlock), 0, s, m,
                         static_cast<int64_t>(L.n_cont) * NR, r, L.L.dinvf.p, L.rf.p, x1, skip);
    const bool widened = bvcycle_level<float, NR>(bt, skip, 0, L.rf.p, L.xf.p, x1 != nullptr, z);
    // rows the last sweep did not write (all rows, or those of single-level
    // systems, which the binary64 solve below overwrites anyway)
    if (!widened) hipLaunchKernelGGL(k_bf2d, rgrid(k_bf2d, m), dim3(kBlock), 0, s, m, L.xf.p, z, skip);
    // single-level systems: their whole cycle is the binary64 direct solve
    if (L.nterm > 0)
      hipLaunchKernelGGL((k_bcoarse<double, NR>), dim3(L.nterm), dim3(kBlock), 0, s, skip,
                         L.term_off.p, L.term_n.p, L.term_inv.p, L.inv_pool.p, r, z);
  } else {
    bvcycle_level<double, NR>(bt, skip, 0, r, z, false);
  }
  AMG_LAUNCH_CHECK();
}

template <int NR, int PC>
void launch_spmm_dots_pc(amg_batch *bt, const int *skip) {
  const BLevel &L0 = bt->B[0];
  auto kern = coded_only(L0.L) ? k_bpcg_spmm_dots<NR, PC, true> : k_bpcg_spmm_dots<NR, PC, false>;
  hipLaunchKernelGGL(kern, rgrid(kern, static_cast<int64_t>(bt->ntiles) * kBlock),
                     dim3(kBlock), 0, bt->stream, skip, bt->ntiles, bt->trow0.p, bt->trow1.p, L0.L.S.sptr.p,
                     L0.L.S.col.p, L0.L.S.val.p, bt->w.p, bt->r.p, bt->q.p, bt->v.p, bt->partials.p,
                     bcodes<double>(L0.L));
}

template <int NR>
void launch_spmm_dots(amg_batch *bt, const int *skip) {
  launch_spmm_dots_pc<NR, spmm_cols<NR>()>(bt, skip);
}

template <int NR>
void launch_update(amg_batch *bt, const int *skip) {
  hipLaunchKernelGGL((k_bpcg_update<NR>), rgrid((k_bpcg_update<NR>), static_cast<int64_t>(bt->ntiles) * kBlock),
                     dim3(kBlock), 0, bt->stream, skip, bt->ntiles, bt->trow0.p, bt->trow1.p, bt->tsys.p,
                     bt->w.p, bt->v.p, bt->d.p, bt->u.p, bt->q.p, bt->r.p, bt->sc.p, bt->partials.p,
                     bfirst_out<NR>(bt));
}

template <int NR>
void benqueue_iteration(amg_batch *bt, int maxit) {
  hipStream_t s = bt->stream;
  const int *skip = bt->all_done.p;
  bvcycle<NR>(bt, skip, bt->r.p, bt->w.p, true);   // r came from the init or the last update
  launch_spmm_dots<NR>(bt, skip);
  hipLaunchKernelGGL((k_bpcg_dots_finish<NR>), dim3(bt->nsys), dim3(kBFinish), 0, s, skip,
                     bt->tile_ptr.p, bt->partials.p, bt->sc.p);
  launch_update<NR>(bt, skip);
  hipLaunchKernelGGL((k_bpcg_norm_finish<NR>), dim3(bt->nsys), dim3(kBFinish), 0, s, skip,
                     bt->tile_ptr.p, bt->partials.p, bt->sc.p, maxit, bt->active.p);
  hipLaunchKernelGGL(k_ball_done, dim3(1), dim3(1), 0, s, bt->active.p, bt->all_done.p,
                     bt->host_flag_dev);
  AMG_LAUNCH_CHECK();
}

// Time the sweep variants on every level with active smoothing rows and keep
// the fastest columns-per-lane (rows per wave = 64 / (NR / cpl)); the
// corrected sweep (which also gathers P values, aggregate ids and the
// coarse correction) is timed and chosen on its own.
// Time of five back-to-back runs of launch() on s, after one warm run.
struct LaunchTimer {
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  explicit LaunchTimer(hipStream_t st) : s(st) {
    AMG_HIP(hipEventCreate(&e0));
    AMG_HIP(hipEventCreate(&e1));
  }
  ~LaunchTimer() {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  LaunchTimer(const LaunchTimer &) = delete;
  LaunchTimer &operator=(const LaunchTimer &) = delete;
  template <class F>
  float operator()(F &&launch) {
    launch();
    AMG_HIP(hipEventRecord(e0, s));
    for (int q = 0; q < 5; ++q) launch();
    AMG_HIP(hipEventRecord(e1, s));
    AMG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  }
};

template <class T, int NR>
void autotune(amg_batch *bt) {
  hipStream_t s = bt->stream;
  LaunchTimer time5(s);
  for (size_t k = 0; k < bt->B.size(); ++k) {
    BLevel &L = bt->B[k];
    L.cpl = L.cpl_corr = 1;
    if (L.n_cont == 0 || NR == 1) continue;
    const int64_t m = static_cast<int64_t>(L.n) * NR;
    T *x = bv_x<T>(L), *t = bv_t<T>(L), *r = bv_r<T>(L);
    for (T *p : {x, t, r}) hipLaunchKernelGGL(k_bzero<T>, rgrid(k_bzero<T>, m), dim3(kBlock), 0, s, m, p);
    T *e = nullptr;
    if (k + 1 < bt->B.size()) {
      const int64_t mc = static_cast<int64_t>(bt->B[k + 1].n) * NR;
      e = bv_x<T>(bt->B[k + 1]);
      hipLaunchKernelGGL(k_bzero<T>, rgrid(k_bzero<T>, mc), dim3(kBlock), 0, s, mc, e);
    }
    float best = 1e30f, best_corr = 1e30f;
    int win_corr = 1, win_wide = 1;
    for (int cpl : {1, 2, 4, 8, 16}) {
      if (NR % cpl != 0) continue;
      L.cpl = L.cpl_corr = cpl;
      const float ms = time5([&] { sweep_any<T, NR>(nullptr, L, L.n_cont, r, x, t, s); });
      if (ms < best) { best = ms; L.tune_best = cpl; }
      if (e) {
        const float mc = time5([&] { corr_sweep_any<T, NR>(nullptr, L, L.n_cont, r, e, x, t, s); });
        if (mc < best_corr) { best_corr = mc; win_corr = cpl; }
      }
    }
    L.cpl = L.tune_best;
    L.cpl_corr = e ? win_corr : L.cpl;
    L.cpl_wide = L.cpl;
    if constexpr (std::is_same<T, float>::value) {
      if (k == 0) {   // the last post-sweep of a binary32 cycle writes binary64 (into w here)
        float best_wide = 1e30f;
        for (int cpl : {1, 2, 4, 8, 16}) {
          if (NR % cpl != 0) continue;
          L.cpl_wide = cpl;
          const float mw = time5([&] { sweep_widen_any<NR>(nullptr, L, L.n_cont, r, x, bt->w.p, s); });
          if (mw < best_wide) { best_wide = mw; win_wide = cpl; }
        }
        L.cpl_wide = win_wide;
      }
    }
  }
}


}  // namespace
}  // namespace amg

namespace amg {
namespace {

// ------------------------------------------------------------ batched setup
int count_tiles(const std::vector<int64_t> &roff0, int tile_rows) {
  int64_t n = 0;
  for (size_t p = 0; p + 1 < roff0.size(); ++p) n += (roff0[p + 1] - roff0[p] + tile_rows - 1) / tile_rows;
  return static_cast<int>(n);
}

// Level-0 reduction tiles of at most tile_rows rows, never crossing a
// system; the device arrays are sized for the largest tile count.
void set_tiles(amg_batch *bt, int tile_rows) {
  hipStream_t s = bt->stream;
  const int nsys = bt->nsys;
  const std::vector<int64_t> &roff0 = bt->roff0;
  std::vector<int> r0, r1, ts, tp(nsys + 1, 0);
  for (int p = 0; p < nsys; ++p) {
    tp[p] = static_cast<int>(r0.size());
    for (int64_t a = roff0[p]; a < roff0[p + 1]; a += tile_rows) {
      r0.push_back(static_cast<int>(a));
      r1.push_back(static_cast<int>(std::min<int64_t>(a + tile_rows, roff0[p + 1])));
      ts.push_back(p);
    }
  }
  tp[nsys] = static_cast<int>(r0.size());
  bt->ntiles = static_cast<int>(r0.size());
  bt->tile_rows = tile_rows;
  if (bt->trow0.n != static_cast<size_t>(bt->max_tiles)) {
    bt->trow0.alloc(bt->max_tiles);
    bt->trow1.alloc(bt->max_tiles);
    bt->tsys.alloc(bt->max_tiles);
  }
  if (bt->tile_ptr.n != static_cast<size_t>(nsys + 1)) bt->tile_ptr.alloc(nsys + 1);
  if (bt->ntiles > 0) {
    AMG_HIP(hipMemcpyAsync(bt->trow0.p, r0.data(), sizeof(int) * bt->ntiles, hipMemcpyHostToDevice, s));
    AMG_HIP(hipMemcpyAsync(bt->trow1.p, r1.data(), sizeof(int) * bt->ntiles, hipMemcpyHostToDevice, s));
    AMG_HIP(hipMemcpyAsync(bt->tsys.p, ts.data(), sizeof(int) * bt->ntiles, hipMemcpyHostToDevice, s));
  }
  AMG_HIP(hipMemcpyAsync(bt->tile_ptr.p, tp.data(), sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, s));
  AMG_HIP(hipStreamSynchronize(s));
}

void batch_build(amg_batch *bt, int nsys, const amg_csr *A) {
  hipStream_t s = bt->stream;
  const bool mixed = bt->p.precision == AMG_PREC_MIXED;
  const double t0 = wall_ms();
  std::vector<amg_hierarchy *> H(nsys, nullptr);
  struct Cleanup {
    std::vector<amg_hierarchy *> &H;
    hipStream_t s;
    ~Cleanup() {
      (void)hipStreamSynchronize(s);   // the copies below read the systems' buffers
      for (auto *h : H)
        if (h) { destroy_graph(h); if (h->sc_host) (void)hipHostFree(h->sc_host); delete h; }
    }
  } cleanup{H, s};
  bt->nsys = nsys;
  bt->nl.assign(nsys, 0);
  bt->n0.assign(nsys, 0);
  if (bt->p.smooth_vec == AMG_SMOOTH_GIVEN) fail(AMG_ERR_UNSUPPORTED, "batched setup takes no given smooth vector");
  // The systems' hierarchies are independent: host threads build them
  // concurrently, each on a library stream of its own (setups are chains of
  // small kernels and host reads, so they overlap well on the GPU).
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  // AMG_BUILD_THREADS (1 .. kBuildThreads) lowers the thread count, e.g.
  // for tools that trace every dispatch of every thread
  int want = kBuildThreads;
  if (const char *env = std::getenv("AMG_BUILD_THREADS")) {
    const int v = std::atoi(env);
    if (v >= 1 && v <= kBuildThreads) want = v;
  }
  const int nthreads = std::max(1, std::min(nsys, want));
  std::atomic<int> next{0};
  std::mutex emu;
  Error first{AMG_OK, ""};
  auto worker = [&](int w) {
    try {
      AMG_HIP(hipSetDevice(dev));
      hipStream_t ws = library_stream(1 + w);
      if (!ws) fail(AMG_ERR_DEVICE, "hipStreamCreate failed");
      PoolScope pool(ws);
      for (int sid = next++; sid < nsys; sid = next++) {
        {
          std::lock_guard<std::mutex> lock(emu);
          if (first.code != AMG_OK) return;
        }
        amg_hierarchy *h = new amg_hierarchy();
        H[sid] = h;
        h->p = bt->p;
        h->p.smooth_vector = nullptr;
        h->p.value_coding = AMG_VALUES_PLAIN;   // the batched kernels read plain values
        h->stream = ws;
        build_hierarchy(h, &A[sid]);
        AMG_HIP(hipStreamSynchronize(ws));
        if (bt->p.precond && !h->coarse_dense)
          fail(AMG_ERR_UNSUPPORTED, "batched solve needs a direct coarsest solve on every system");
      }
    } catch (const Error &e) {
      std::lock_guard<std::mutex> lock(emu);
      if (first.code == AMG_OK) first = e;
    } catch (const std::bad_alloc &) {
      std::lock_guard<std::mutex> lock(emu);
      if (first.code == AMG_OK) first = Error{AMG_ERR_NOMEM, "host allocation failed"};
    } catch (...) {
      std::lock_guard<std::mutex> lock(emu);
      if (first.code == AMG_OK) first = Error{AMG_ERR_DEVICE, "unexpected error in a setup thread"};
    }
  };
  {
    std::vector<std::thread> pool;
    for (int w = 1; w < nthreads; ++w) pool.emplace_back(worker, w);
    worker(0);
    for (std::thread &th : pool) th.join();
  }
  if (first.code != AMG_OK) fail(first.code, first.msg);
  bt->p.model_params = nullptr;
  bt->p.model_path = nullptr;
  // deepest systems first (stable): active systems on any level form a prefix
  std::vector<int> order(nsys);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return H[a]->L.size() > H[b]->L.size(); });
  bt->order = order;
  bt->pos_of.assign(nsys, 0);
  std::vector<int> nlp(nsys);
  for (int p = 0; p < nsys; ++p) { bt->pos_of[order[p]] = p; nlp[p] = static_cast<int>(H[order[p]]->L.size()); }
  for (int sid = 0; sid < nsys; ++sid) { bt->nl[sid] = static_cast<int>(H[sid]->L.size()); bt->n0[sid] = H[sid]->L[0].A.n; }
  const int max_nl = nlp[0];
  bt->B.clear();
  bt->B.resize(max_nl);
  std::vector<int64_t> roff0;
  for (int k = 0; k < max_nl; ++k) {
    BLevel &BL = bt->B[k];
    int na = 0, ncnt = 0;
    while (na < nsys && nlp[na] > k) ++na;
    while (ncnt < na && nlp[ncnt] > k + 1) ++ncnt;
    std::vector<int64_t> roff(na + 1, 0), zoff(na + 1, 0);
    for (int p = 0; p < na; ++p) {
      const Level &Ls = H[order[p]]->L[k];
      roff[p + 1] = roff[p] + Ls.A.n;
      zoff[p + 1] = zoff[p] + Ls.A.nnz;
    }
    if (roff[na] >= (int64_t(1) << 31) / 16 || zoff[na] >= (int64_t(1) << 31))
      fail(AMG_ERR_UNSUPPORTED, "batched problem too large for int32 indexing");
    if (k == 0) roff0 = roff;
    BL.n = static_cast<int>(roff[na]);
    BL.n_cont = static_cast<int>(roff[ncnt]);
    DevCSR &C = BL.L.A;
    C.n = BL.n;
    C.nnz = zoff[na];
    C.rp.alloc(C.n + 1);
    C.ci.alloc(C.nnz);
    C.v.alloc(C.nnz);
    for (int p = 0; p < na; ++p) {
      const Level &Ls = H[order[p]]->L[k];
      hipLaunchKernelGGL(k_add_copy, grid_for(Ls.A.n), dim3(kBlock), 0, s, Ls.A.n, Ls.A.rp.p,
                         C.rp.p + roff[p], static_cast<int>(zoff[p]));
      hipLaunchKernelGGL(k_add_copy, grid_for(Ls.A.nnz), dim3(kBlock), 0, s, static_cast<int>(Ls.A.nnz),
                         Ls.A.ci.p, C.ci.p + zoff[p], static_cast<int>(roff[p]));
      AMG_HIP(hipMemcpyAsync(C.v.p + zoff[p], Ls.A.v.p, sizeof(double) * Ls.A.nnz,
                             hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(k_set_one, dim3(1), dim3(1), 0, s, C.rp.p + C.n, static_cast<int>(C.nnz));
    AMG_LAUNCH_CHECK();
    finalize_level(BL.L, s, mixed, true);
    if (ncnt > 0 && k + 1 < max_nl) {
      std::vector<int64_t> coff(ncnt + 1, 0);
      for (int p = 0; p < ncnt; ++p) coff[p + 1] = coff[p] + H[order[p]]->L[k + 1].A.n;
      Level &L = BL.L;
      L.nc = static_cast<int>(coff[ncnt]);
      L.agg.alloc(BL.n_cont);
      L.pval.alloc(BL.n_cont);
      if (mixed) L.pvalf.alloc(BL.n_cont);
      L.mptr.alloc(L.nc + 1);
      L.mem.alloc(BL.n_cont);
      for (int p = 0; p < ncnt; ++p) {
        const Level &Ls = H[order[p]]->L[k];
        const int nk = Ls.A.n, nck = Ls.nc;
        hipLaunchKernelGGL(k_add_copy, grid_for(nk), dim3(kBlock), 0, s, nk, Ls.agg.p, L.agg.p + roff[p],
                           static_cast<int>(coff[p]));
        AMG_HIP(hipMemcpyAsync(L.pval.p + roff[p], Ls.pval.p, sizeof(double) * nk, hipMemcpyDeviceToDevice, s));
        if (mixed)
          AMG_HIP(hipMemcpyAsync(L.pvalf.p + roff[p], Ls.pvalf.p, sizeof(float) * nk,
                                 hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_add_copy, grid_for(nck), dim3(kBlock), 0, s, nck, Ls.mptr.p, L.mptr.p + coff[p],
                           static_cast<int>(roff[p]));
        hipLaunchKernelGGL(k_add_copy, grid_for(nk), dim3(kBlock), 0, s, nk, Ls.mem.p, L.mem.p + roff[p],
                           static_cast<int>(roff[p]));
      }
      hipLaunchKernelGGL(k_set_one, dim3(1), dim3(1), 0, s, L.mptr.p + L.nc, BL.n_cont);
      AMG_LAUNCH_CHECK();
    }
    // systems whose coarsest level is k
    BL.nterm = na - ncnt;
    if (BL.nterm > 0) {
      std::vector<int> toff, tn;
      std::vector<long long> tinv;
      long long pool = 0;
      for (int p = ncnt; p < na; ++p) {
        const int m = H[order[p]]->L[k].A.n;
        toff.push_back(static_cast<int>(roff[p]));
        tn.push_back(m);
        tinv.push_back(pool);
        pool += static_cast<long long>(m) * m;
      }
      BL.term_off.alloc(BL.nterm);
      BL.term_n.alloc(BL.nterm);
      BL.term_inv.alloc(BL.nterm);
      BL.inv_pool.alloc(std::max<long long>(1, pool));
      AMG_HIP(hipMemcpyAsync(BL.term_off.p, toff.data(), sizeof(int) * BL.nterm, hipMemcpyHostToDevice, s));
      AMG_HIP(hipMemcpyAsync(BL.term_n.p, tn.data(), sizeof(int) * BL.nterm, hipMemcpyHostToDevice, s));
      AMG_HIP(hipMemcpyAsync(BL.term_inv.p, tinv.data(), sizeof(long long) * BL.nterm, hipMemcpyHostToDevice, s));
      for (int p = ncnt, q = 0; p < na; ++p, ++q) {
        const amg_hierarchy *hs = H[order[p]];
        const int m = tn[q];
        if (bt->p.precond)
          AMG_HIP(hipMemcpyAsync(BL.inv_pool.p + tinv[q], hs->Ainv.p, sizeof(double) * m * m,
                                 hipMemcpyDeviceToDevice, s));
      }
      AMG_HIP(hipStreamSynchronize(s));
    }
    AMG_HIP(hipStreamSynchronize(s));
  }
  // level-0 tiles (never crossing a system) and row offsets
  bt->roff0 = roff0;
  bt->max_tiles = 0;
  bt->max_tiles = count_tiles(roff0, kBTile);
  set_tiles(bt, kBTile);
  bt->user_off.assign(nsys + 1, 0);
  bt->int_off.assign(nsys, 0);
  for (int sid = 0; sid < nsys; ++sid) {
    bt->user_off[sid + 1] = bt->user_off[sid] + bt->n0[sid];
    bt->int_off[sid] = roff0[bt->pos_of[sid]];
  }
  bt->nnz0 = bt->B[0].L.A.nnz;
  AMG_HIP(hipStreamSynchronize(s));
  bt->setup_ms = wall_ms() - t0;
}

void batch_release_graph(amg_batch *bt) {
  if (bt->graph_exec) (void)hipGraphExecDestroy(bt->graph_exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->graph_exec = nullptr;
  bt->graph = nullptr;
}

template <int NR>
void batch_buffers(amg_batch *bt) {
  if (bt->nr == NR) return;
  batch_release_graph(bt);
  const bool mixed = bt->p.precision == AMG_PREC_MIXED;
  for (auto &L : bt->B) {
    const size_t m = static_cast<size_t>(L.n) * NR;
    if (mixed) { L.rf.alloc(m); L.xf.alloc(m); L.tf.alloc(m); L.r.release(); L.x.release(); L.t.release(); }
    else { L.r.alloc(m); L.x.alloc(m); L.t.alloc(m); L.rf.release(); L.xf.release(); L.tf.release(); }
  }
  const size_t m0 = static_cast<size_t>(bt->B[0].n) * NR;
  for (auto *v : {&bt->bint, &bt->u, &bt->r, &bt->w, &bt->v, &bt->d, &bt->q}) v->alloc(m0);
  bt->partials.alloc(static_cast<size_t>(bt->max_tiles) * NR * 3);
  bt->sc.alloc(static_cast<size_t>(bt->nsys) * NR);
  bt->active.alloc(1);
  bt->all_done.alloc(1);
  if (!bt->host_flag) {
    AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&bt->host_flag), sizeof(int),
                          hipHostMallocMapped | hipHostMallocCoherent));
    AMG_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&bt->host_flag_dev), bt->host_flag, 0));
  }
  const double t0 = wall_ms();
  if (bt->p.precond) {
    if (mixed) autotune<float, NR>(bt);
    else autotune<double, NR>(bt);
  }
  bt->spmm_cols = spmm_cols<NR>();
  AMG_HIP(hipStreamSynchronize(bt->stream));
  bt->tune_ms = wall_ms() - t0;
  bt->nr = NR;
}

// The caller's vectors: one block with the systems one after another
// (base), or one pointer per system (each, in the order of amg_batch_setup).
struct UserVecs {
  const double *base = nullptr;
  const double *const *each = nullptr;
  double *at(const amg_batch *bt, int sid, int nr) const {
    return const_cast<double *>(each ? each[sid] : base + bt->user_off[sid] * nr);
  }
};

// user layout (systems in user order) <-> internal layout (depth order)
template <int NR>
void batch_permute(amg_batch *bt, const UserVecs &user, double *internal, bool to_internal) {
  for (int sid = 0; sid < bt->nsys; ++sid) {
    const int64_t ii = bt->int_off[sid] * NR, m = bt->n0[sid] * NR;
    double *u = user.at(bt, sid, NR);
    if (to_internal)
      AMG_HIP(hipMemcpyAsync(internal + ii, u, sizeof(double) * m, hipMemcpyDeviceToDevice, bt->stream));
    else
      AMG_HIP(hipMemcpyAsync(u, internal + ii, sizeof(double) * m, hipMemcpyDeviceToDevice, bt->stream));
  }
}

// Iterations per graph launch.  Iterations launched after every pair has
// converged still dispatch all their kernels (about 73 at 64 x 16, 0.2-0.3 ms
// an iteration), so launches are short: 64 x 16 solve 0.1719 s with 32
// (20 such iterations), 0.1698 s with 1, 2 or 4.
#ifndef AMG_BATCH_GRAPH_ITERS
#define AMG_BATCH_GRAPH_ITERS 2
#endif
constexpr int kGraphIters = AMG_BATCH_GRAPH_ITERS;

template <int NR>
int batch_solve_nr(amg_batch *bt, const UserVecs &Bu, const UserVecs &Xu, double rtol, int maxit,
                   int32_t *iters, double *relres, int32_t *status) {
  hipStream_t s = bt->stream;
  batch_buffers<NR>(bt);
  const int64_t m0 = static_cast<int64_t>(bt->B[0].n) * NR;
  const BLevel &L0 = bt->B[0];
  batch_permute<NR>(bt, Bu, bt->bint.p, true);
  batch_permute<NR>(bt, Xu, bt->u.p, true);
  hipLaunchKernelGGL(k_bzero<double>, rgrid(k_bzero<double>, m0), dim3(kBlock), 0, s, m0, bt->d.p);
  hipLaunchKernelGGL(k_bzero<double>, rgrid(k_bzero<double>, m0), dim3(kBlock), 0, s, m0, bt->q.p);
  AMG_HIP(hipMemsetAsync(bt->active.p, 0, sizeof(int), s));
  hipLaunchKernelGGL((k_bpcg_init<NR>), dim3(bt->ntiles), dim3(kBlock), 0, s, bt->trow0.p, bt->trow1.p,
                     L0.L.S.sptr.p, L0.L.S.col.p, L0.L.S.val.p, bt->bint.p, bt->u.p, bt->r.p,
                     bt->partials.p, bcodes<double>(L0.L), bfirst_out<NR>(bt));
  hipLaunchKernelGGL((k_bpcg_init_finish<NR>), dim3(bt->nsys), dim3(kBFinish), 0, s, bt->tile_ptr.p,
                     bt->partials.p, bt->sc.p, rtol, bt->active.p);
  hipLaunchKernelGGL(k_ball_done, dim3(1), dim3(1), 0, s, bt->active.p, bt->all_done.p, bt->host_flag_dev);
  AMG_LAUNCH_CHECK();
  const int reps = std::min(maxit, kGraphIters);
  if (!bt->graph_exec || bt->graph_reps != reps || bt->graph_maxit != maxit) {
    batch_release_graph(bt);
    capture_graph(bt->stream, &bt->graph, [&] {
      for (int i = 0; i < reps; ++i) benqueue_iteration<NR>(bt, maxit);
    });
    AMG_HIP(hipGraphInstantiate(&bt->graph_exec, bt->graph, nullptr, nullptr, 0));
    bt->graph_reps = reps;
    bt->graph_maxit = maxit;
  }
  AMG_HIP(hipStreamSynchronize(s));
  for (int done_it = 0; !*static_cast<volatile int *>(bt->host_flag) && done_it < maxit; done_it += reps) {
    AMG_HIP(hipGraphLaunch(bt->graph_exec, s));
    AMG_HIP(hipStreamSynchronize(s));
  }
  batch_permute<NR>(bt, Xu, bt->u.p, false);
  std::vector<BScalars> S(static_cast<size_t>(bt->nsys) * NR);
  AMG_HIP(hipMemcpyAsync(S.data(), bt->sc.p, sizeof(BScalars) * S.size(), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  int worst = AMG_OK;
  for (int sid = 0; sid < bt->nsys; ++sid) {
    const int p = bt->pos_of[sid];
    for (int c = 0; c < NR; ++c) {
      const BScalars &x = S[static_cast<size_t>(p) * NR + c];
      const size_t o = static_cast<size_t>(sid) * NR + c;
      iters[o] = x.it;
      relres[o] = (x.nr0 == 0.0) ? 0.0 : sqrt(x.rr) / x.nr0;
      int st = x.status != 0 ? x.status : ((x.conv || x.nr0 == 0.0) ? AMG_OK : AMG_NOT_CONVERGED);
      status[o] = st;
      if (st < 0 && (worst >= 0 || st < worst)) worst = st;
      else if (st == AMG_NOT_CONVERGED && worst == AMG_OK) worst = st;
    }
  }
  return worst;
}

template <int NR>
void batch_vcycle_nr(amg_batch *bt, const UserVecs &Ru, const UserVecs &Zu) {
  batch_buffers<NR>(bt);
  batch_permute<NR>(bt, Ru, bt->r.p, true);
  bvcycle<NR>(bt, nullptr, bt->r.p, bt->w.p);
  batch_permute<NR>(bt, Zu, bt->w.p, false);
  AMG_HIP(hipStreamSynchronize(bt->stream));
}

}  // namespace
}  // namespace amg

namespace amg {
namespace {

int batch_solve_any(amg_batch *bt, int32_t nrhs, const UserVecs &B, const UserVecs &X, double rtol,
                    int32_t maxit, int32_t *iters, double *relres, int32_t *status) {
  return api_guarded([&] {
    switch (nrhs) {
      case 1: return amg::batch_solve_nr<1>(bt, B, X, rtol, maxit, iters, relres, status);
      case 2: return amg::batch_solve_nr<2>(bt, B, X, rtol, maxit, iters, relres, status);
      case 4: return amg::batch_solve_nr<4>(bt, B, X, rtol, maxit, iters, relres, status);
      case 8: return amg::batch_solve_nr<8>(bt, B, X, rtol, maxit, iters, relres, status);
      case 16: return amg::batch_solve_nr<16>(bt, B, X, rtol, maxit, iters, relres, status);
      default: return amg::api_set_error(AMG_ERR_UNSUPPORTED, "nrhs must be 1, 2, 4, 8 or 16");
    }
  });
}

}  // namespace
}  // namespace amg

// ============================================================== C ABI
extern "C" {

int amg_batch_setup(int32_t nsys, const amg_csr *A, const amg_params *p, amg_batch **out) {
  if (out) *out = nullptr;
  if (nsys < 1 || !A || !p || !out) return amg::api_set_error(AMG_ERR_INVALID, "bad argument");
  for (int s = 0; s < nsys; ++s)
    if (A[s].n <= 0 || A[s].nnz < A[s].n || !A[s].row_ptr || !A[s].col_idx || !A[s].val)
      return amg::api_set_error(AMG_ERR_INVALID, "bad CSR header in the batch");
  const int pst = amg::api_check_params(p);
  if (pst != AMG_OK) return pst;
  if (p->max_hrc != 1 || p->cycle_type != AMG_CYCLE_V || p->relax_type != AMG_RELAX_L1_JACOBI ||
      p->coarse_relax != AMG_RELAX_L1_JACOBI)
    return amg::api_set_error(AMG_ERR_UNSUPPORTED, "the batched solve runs the l1-Jacobi V-cycle of one hierarchy");
  amg_batch *bt = new (std::nothrow) amg_batch();
  if (!bt) return amg::api_set_error(AMG_ERR_NOMEM, "host allocation failed");
  bt->p = *p;
  bt->p.smooth_vector = nullptr;   // (model_params / model_path stay valid while amg_batch_setup runs)
  if (p->stream) {
    bt->stream = static_cast<hipStream_t>(p->stream);
  } else {
    bt->stream = amg::acquire_private_stream(&bt->stream_dev);
    if (!bt->stream) {
      delete bt;
      return amg::api_set_error(AMG_ERR_DEVICE, "no HIP device or stream available (hipGetDevice / hipStreamCreate failed)");
    }
    bt->own_stream = true;
  }
  int st = amg::api_guarded([&] {
    amg::keep_pool_memory();
    amg::SetupStream on(bt->stream, !bt->own_stream);
    amg::PoolScope pool(bt->stream);
    amg::batch_build(bt, nsys, A);
    return AMG_OK;
  });
  if (st != AMG_OK) {
    std::string msg = amg::api_last_error();
    amg_batch_destroy(bt);
    amg::api_set_error(st, msg);
    return st;
  }
  *out = bt;
  return AMG_OK;
}


int amg_batch_solve(amg_batch *bt, int32_t nrhs, const double *B, double *X, double rtol,
                    int32_t maxit, int32_t *iters, double *relres, int32_t *status) {
  if (!bt || !B || !X || !iters || !relres || !status || !(rtol > 0.0) || maxit < 1)
    return amg::api_set_error(AMG_ERR_INVALID, "bad argument");
  amg::UserVecs b, x;
  b.base = B;
  x.base = X;
  return amg::batch_solve_any(bt, nrhs, b, x, rtol, maxit, iters, relres, status);
}

int amg_batch_solve_systems(amg_batch *bt, int32_t nrhs, const double *const *B, double *const *X,
                            double rtol, int32_t maxit, int32_t *iters, double *relres,
                            int32_t *status) {
  if (!bt || !B || !X || !iters || !relres || !status || !(rtol > 0.0) || maxit < 1)
    return amg::api_set_error(AMG_ERR_INVALID, "bad argument");
  for (int sid = 0; sid < bt->nsys; ++sid)
    if (!B[sid] || !X[sid]) return amg::api_set_error(AMG_ERR_INVALID, "NULL system vector");
  amg::UserVecs b, x;
  b.each = B;
  x.each = X;
  return amg::batch_solve_any(bt, nrhs, b, x, rtol, maxit, iters, relres, status);
}

int amg_batch_vcycle(amg_batch *bt, int32_t nrhs, const double *R, double *Z) {
  if (!bt || !R || !Z || R == Z) return amg::api_set_error(AMG_ERR_INVALID, "bad argument");
  amg::UserVecs r, z;
  r.base = R;
  z.base = Z;
  return amg::api_guarded([&] {
    switch (nrhs) {
      case 1: amg::batch_vcycle_nr<1>(bt, r, z); break;
      case 2: amg::batch_vcycle_nr<2>(bt, r, z); break;
      case 4: amg::batch_vcycle_nr<4>(bt, r, z); break;
      case 8: amg::batch_vcycle_nr<8>(bt, r, z); break;
      case 16: amg::batch_vcycle_nr<16>(bt, r, z); break;
      default: return amg::api_set_error(AMG_ERR_UNSUPPORTED, "nrhs must be 1, 2, 4, 8 or 16");
    }
    return AMG_OK;
  });
}

int amg_batch_info(const amg_batch *bt, amg_batch_info_t *out) {
  if (!bt || !out) return amg::api_set_error(AMG_ERR_INVALID, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->nsys = bt->nsys;
  out->levels = static_cast<int32_t>(bt->B.size());
  for (size_t k = 0; k < bt->B.size() && k < AMG_MAX_LEVELS; ++k) {
    out->n[k] = bt->B[k].n;
    out->n_smoothed[k] = bt->B[k].n_cont;
    out->nnz[k] = bt->B[k].L.A.nnz;
    out->cols_per_lane[k] = bt->B[k].cpl;
    out->cols_per_lane_corr[k] = bt->B[k].cpl_corr;
  }
  out->tile_rows = bt->tile_rows;
  out->spmm_cols = bt->spmm_cols;
  out->setup_ms = bt->setup_ms;
  out->tune_ms = bt->tune_ms;
  return AMG_OK;
}

void amg_batch_destroy(amg_batch *bt) {
  if (!bt) return;
  (void)hipStreamSynchronize(bt->stream);
  amg::batch_release_graph(bt);
  if (bt->host_flag) (void)hipHostFree(bt->host_flag);
  const bool own = bt->own_stream;
  const int dev = bt->stream_dev;
  hipStream_t s = bt->stream;
  {
    amg::FreeOn on(amg::library_stream());   // bt->stream is idle and may be the caller's
    delete bt;
  }
  if (own) amg::release_private_stream(dev, s);
}

}  // extern "C"
