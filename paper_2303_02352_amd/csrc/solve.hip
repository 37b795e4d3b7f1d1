// Solve phase: V-cycle (Alg. 2) and flexible PCG (Alg. 1) on the GPU.
//
// Matrices are read in the SELL-64 layout (one wavefront of rows per slice,
// one row per lane, entries in CSR order), so every row sum is a left fold
// in CSR order: SpMV, sweeps, residuals, restriction and prolongation give
// the same bits as a sequential evaluation.  Only the three PCG dot products
// and the residual norm are tree reductions; they run in two phases (one
// partial per workgroup, then one workgroup folds the partials in index
// order), so they are repeatable and need no grid-wide fences.
//
// Kernels that belong to a PCG iteration take `skip` (the device-side
// `done` flag): once the iteration has converged or broken down they return
// at once, which lets the host keep the next iteration queued.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "amg_internal.hpp"

namespace amg {

namespace {

inline dim3 grid_for(int64_t n, int block = kBlock) {
  return dim3(static_cast<unsigned>(std::max<int64_t>(1, (n + block - 1) / block)));
}

#define AMG_SKIP_IF_DONE() \
  if (skip && *skip) return

// Eight wavefronts per SIMD for the streaming row kernels: the register
// budget this sets (64 VGPRs, from about 70) costs nothing and the eighth
// wavefront adds loads in flight (fine sweep 68.5 -> 67.6 us).
#define AMG_EIGHT_WAVES __attribute__((amdgpu_waves_per_eu(8)))

// ------------------------------------------------------ SELL row kernels
// Row r of slice s: slots sptr[s] + k*64 + lane, k < width(s).  Streamed
// (non-temporal) loads for matrices read once per pass; plain loads in the
// coarse-tail kernel, whose working set stays in cache.
// Fold of one SELL row: slots k = 0 .. width-1 in order, acc += a_k x(c_k),
// l1 += |a_k|.  Slots are taken eight at a time (two quads), the last 1-7
// in one predicated batch (width is the same on the whole wavefront), so all
// loads of a batch are in flight together.  Column and value sources fill
// one quad of slots at a time: load4(t, nv, out) sets out[j] for slot
// 4t + j, j < nv.
template <class T, bool kStream, class Cols, class Vals, class G>
__device__ __forceinline__ void row_fold(Cols cols, Vals vals, G x, int width, T &sum, T &l1) {
  T acc = T(0), m = T(0);
  int t = 0;
  for (; 4 * t + 8 <= width; t += 2) {
    int c0[4], c1[4];
    T a0[4], a1[4], x0[4], x1[4];
    cols.load4(t, 4, c0);
    cols.load4(t + 1, 4, c1);
    vals.load4(t, 4, a0);
    vals.load4(t + 1, 4, a1);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x0[u] = x(c0[u]);
      x1[u] = x(c1[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc = acc + a0[u] * x0[u];
      m = m + fabs(a0[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc = acc + a1[u] * x1[u];
      m = m + fabs(a1[u]);
    }
  }
  const int rem = width - 4 * t;
  if (rem > 0) {
    const int n0 = rem < 4 ? rem : 4, n1 = rem - n0;
    int c0[4], c1[4];
    T a0[4], a1[4], x0[4], x1[4];
    cols.load4(t, n0, c0);
    vals.load4(t, n0, a0);
    if (n1 > 0) {
      cols.load4(t + 1, n1, c1);
      vals.load4(t + 1, n1, a1);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < n0) x0[u] = x(c0[u]);
      if (u < n1) x1[u] = x(c1[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (u < n0) {
        acc = acc + a0[u] * x0[u];
        m = m + fabs(a0[u]);
      }
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (u < n1) {
        acc = acc + a1[u] * x1[u];
        m = m + fabs(a1[u]);
      }
  }
  sum = acc;
  l1 = m;
}

template <class V, bool kStream>
__device__ __forceinline__ V ldx(const V *p) {
  return kStream ? ld_stream(p) : *p;
}

template <bool kStream>
struct PlainCols {      // int32 column of slot k (slot-major layout)
  const int *__restrict__ cp;
  __device__ __forceinline__ void load4(int t, int nv, int (&c)[4]) const {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nv) c[j] = ldx<int, kStream>(cp + (4 * t + j) * 64);
  }
};

template <bool kStream>
struct QuadCols {       // group base + 16-bit offset, four slots per load
  const int *__restrict__ bp;                  // cbase of the slice's first group
  const unsigned long long *__restrict__ dq;   // the lane's first quad
  __device__ __forceinline__ void load4(int t, int nv, int (&c)[4]) const {
    const unsigned long long d = ldx<unsigned long long, kStream>(dq + t * 64);
    int base[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) base[j] = bp[4 * t + j];   // in range: cbase is padded
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nv) c[j] = base[j] + static_cast<int>((d >> (16 * j)) & 0xffffu);
  }
};

template <class T, bool kStream>
struct PlainVals {      // binary64 / binary32 value of slot k (slot-major layout)
  const T *__restrict__ vp;
  __device__ __forceinline__ void load4(int t, int nv, T (&a)[4]) const {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nv) a[j] = ldx<T, kStream>(vp + (4 * t + j) * 64);
  }
};

template <class T, bool kStream>
struct QuadCodedVals {  // table entries named by the four code bytes of a quad
  const unsigned *__restrict__ cq;   // the lane's first quad
  const T *dict;                     // the table, staged in LDS
  __device__ __forceinline__ void load4(int t, int nv, T (&a)[4]) const {
    const unsigned w = ldx<unsigned, kStream>(cq + t * 64);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nv) a[j] = dict[(w >> (8 * j)) & 0xffu];
  }
};

// Device-side view of a matrix's values.  For a coded matrix each
// wavefront keeps its own copy of the value table in LDS (sdict holds
// kDictMax entries per wavefront): a table of at most 64 entries is loaded
// one entry per lane into a register when the kernel starts and written to
// LDS (publish) only before the first lookup, so its load overlaps the first
// loads of the rows; a larger table is copied at once.  A wavefront's LDS
// accesses complete in issue order, so no workgroup barrier is needed.
template <class T>
struct ValDev {
  const T *val;
  const unsigned char *code;   // null: read val
  T *mine;                     // this wavefront's table in LDS
  T reg;                       // entry `lane` of a small table
  int ndict;
  __device__ __forceinline__ void publish() const {
    if (code && ndict <= kWave) {   // uniform
      const int lane = threadIdx.x & (kWave - 1);
      if (lane < ndict) mine[lane] = reg;
      __builtin_amdgcn_wave_barrier();
    }
  }
};

template <class T>
__device__ __forceinline__ ValDev<T> stage_dict(const ValRef<T> &V, T *sdict) {
  ValDev<T> D{V.val, V.code, nullptr, T(0), V.ndict};
  if (!V.code) return D;   // uniform: a kernel argument
  const int lane = threadIdx.x & (kWave - 1);
  D.mine = sdict + (threadIdx.x / kWave) * kDictMax;
  if (V.ndict <= kWave) {
    D.reg = V.dict[lane < V.ndict ? lane : 0];
  } else {
    for (int i = lane; i < V.ndict; i += kWave) D.mine[i] = V.dict[i];
    __builtin_amdgcn_wave_barrier();
  }
  return D;
}

template <class T>
struct Plain {          // x_c
  const T *__restrict__ x;
  __device__ __forceinline__ T operator()(int c) const { return x[c]; }
};

template <class T>
struct Corrected {      // (x + P e)_c = x_c + p_c e[agg_c], the prolongation's value
  const T *__restrict__ x;
  const T *__restrict__ pval;
  const int *__restrict__ agg;
  const T *__restrict__ e;
  __device__ __forceinline__ T operator()(int c) const { return x[c] + pval[c] * e[agg[c]]; }
};

// Row r through the compact column form (16-bit offsets from a per-group
// base) where its slice has one, else the int32 columns; values plain or
// coded.  The rows of a wavefront must lie in one slice (rows are handed out
// in whole slices), so the slice bounds and group bases are wavefront-uniform
// and read with scalar loads.  Every combination folds the same terms in the
// same order: identical bits.
template <class T, bool kStream, class G>
__device__ __forceinline__ void sell_row_g(const SellRef &S, const ValDev<T> &V, G x, int r, T &sum,
                                           T &l1) {
  const int s = __builtin_amdgcn_readfirstlane(r >> 6);
  const int b = S.sptr[s], width = (S.sptr[s + 1] - b) >> 6;
  const int g = b >> 6;
  const int lane = r & 63;
  const bool compact = S.cdel && width > 0 && S.cbase[g] >= 0;
  const int q = S.qptr[s];
  const int64_t lq = static_cast<int64_t>(q) * 64 + lane;   // the lane's first quad
  const QuadCols<kStream> qcols{S.cbase + g, reinterpret_cast<const unsigned long long *>(S.cdel) + lq};
  const PlainCols<kStream> pcols{S.col + b + lane};
  if (V.code) {   // V.publish() has run on the whole wavefront
    const QuadCodedVals<T, kStream> vals{reinterpret_cast<const unsigned *>(V.code) + lq, V.mine};
    if (compact) row_fold<T, kStream>(qcols, vals, x, width, sum, l1);
    else row_fold<T, kStream>(pcols, vals, x, width, sum, l1);
  } else {
    const PlainVals<T, kStream> vals{V.val + b + lane};
    if (compact) row_fold<T, kStream>(qcols, vals, x, width, sum, l1);
    else row_fold<T, kStream>(pcols, vals, x, width, sum, l1);
  }
}

template <class T, bool kStream = true>
__device__ __forceinline__ void sell_row(const SellRef &S, const ValDev<T> &V,
                                         const T *__restrict__ x, int r, T &sum, T &l1) {
  sell_row_g<T, kStream>(S, V, Plain<T>{x}, r, sum, l1);
}

// The fold of two rows of one lane, in slices sa and sb (wavefront-uniform),
// both compact and coded with 1 to 8 slots, from their group bases: column
// offsets and codes of both rows, then the iterate at every slot, all in
// flight before the first use (twice the loads per wavefront of one row).
// Slots past a row's width are read at clamped, in-range places and left
// out of the fold, so the fold is the one of row_fold.
template <class T, bool kStream, class G>
__device__ __forceinline__ void fold2_bases(const ValDev<T> &V, const SellRef &S, G x, int sa, int sb,
                                            int lane, int wa, int wb, int qsa, int qsb,
                                            const int (&basea)[8], const int (&baseb)[8], T &sum0,
                                            T &l10, T &sum1, T &l11) {
  const unsigned long long *cd = reinterpret_cast<const unsigned long long *>(S.cdel);
  const unsigned *cc = reinterpret_cast<const unsigned *>(V.code);
  const int64_t qa = static_cast<int64_t>(qsa) * 64 + lane;
  const int64_t qb = static_cast<int64_t>(qsb) * 64 + lane;
  const int ta = wa > 4 ? 64 : 0, tb = wb > 4 ? 64 : 0;   // second quad, or the first again
  const unsigned long long da0 = ldx<unsigned long long, kStream>(cd + qa);
  const unsigned long long da1 = ldx<unsigned long long, kStream>(cd + qa + ta);
  const unsigned long long db0 = ldx<unsigned long long, kStream>(cd + qb);
  const unsigned long long db1 = ldx<unsigned long long, kStream>(cd + qb + tb);
  const unsigned ka0 = ldx<unsigned, kStream>(cc + qa), ka1 = ldx<unsigned, kStream>(cc + qa + ta);
  const unsigned kb0 = ldx<unsigned, kStream>(cc + qb), kb1 = ldx<unsigned, kStream>(cc + qb + tb);
  const int rowa = sa * 64, rowb = sb * 64;   // in-range stand-ins for unused slots (rows < n)
  int ca[8], cb[8];
  T xa[8], xb[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const unsigned long long dA = j < 4 ? da0 : da1, dB = j < 4 ? db0 : db1;
    const int offA = static_cast<int>((dA >> (16 * (j & 3))) & 0xffffu);
    const int offB = static_cast<int>((dB >> (16 * (j & 3))) & 0xffffu);
    ca[j] = j < wa ? basea[j] + offA : rowa;
    cb[j] = j < wb ? baseb[j] + offB : rowb;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    xa[j] = x(ca[j]);
    xb[j] = x(cb[j]);
  }
  V.publish();
  T acc0 = T(0), m0 = T(0), acc1 = T(0), m1 = T(0);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const unsigned kA = j < 4 ? ka0 : ka1, kB = j < 4 ? kb0 : kb1;
    const T aA = V.mine[(kA >> (8 * (j & 3))) & 0xffu];
    const T aB = V.mine[(kB >> (8 * (j & 3))) & 0xffu];
    if (j < wa) {
      acc0 = acc0 + aA * xa[j];
      m0 = m0 + fabs(aA);
    }
    if (j < wb) {
      acc1 = acc1 + aB * xb[j];
      m1 = m1 + fabs(aB);
    }
  }
  sum0 = acc0;
  l10 = m0;
  sum1 = acc1;
  l11 = m1;
}

// fold2_bases where it applies (both slices compact and coded, 1 to 8
// slots); returns false (nothing done) otherwise.
template <class T, bool kStream, class G>
__device__ __forceinline__ bool fold2_short(const SellRef &S, const ValDev<T> &V, G x, int sa, int sb,
                                            int lane, T &sum0, T &l10, T &sum1, T &l11) {
  if (!V.code || !S.cdel) return false;
  // every scalar read first (slice bounds, quad offsets, then the 8 group
  // bases of each slice, in range through the padding), the tests after
  const int ba = S.sptr[sa], ea = S.sptr[sa + 1], bb = S.sptr[sb], eb = S.sptr[sb + 1];
  const int qsa = S.qptr[sa], qsb = S.qptr[sb];
  const int wa = (ea - ba) >> 6, wb = (eb - bb) >> 6;
  const int ga = ba >> 6, gb = bb >> 6;
  int basea[8], baseb[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    basea[j] = S.cbase[ga + j];
    baseb[j] = S.cbase[gb + j];
  }
  if (wa < 1 || wb < 1 || wa > 8 || wb > 8) return false;
  if (basea[0] < 0 || baseb[0] < 0) return false;
  fold2_bases<T, kStream>(V, S, x, sa, sb, lane, wa, wb, qsa, qsb, basea, baseb, sum0, l10, sum1, l11);
  return true;
}

template <class T, bool kStream>
__global__ void __launch_bounds__(kBlock) AMG_EIGHT_WAVES k_spmv(int n, SellRef S, ValRef<T> vref,
                                                 const T *__restrict__ x, T *__restrict__ y) {
  __shared__ T sdict[kDictMax * (kBlock / kWave)];
  const ValDev<T> val = stage_dict(vref, sdict);
  val.publish();   // before any lane leaves
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r >= n) return;
  T s, m;
  sell_row<T, kStream>(S, val, x, r, s, m);
  y[r] = s;
}

// l1-Jacobi sweep: xn = x + dinv * (r - A x), dinv = 1 / sum_j |a_ij| taken
// from the streamed row (the same fold that defines the stored diagonal).
// xw: when not null the new iterate is stored there widened to binary64
// instead of in xn (the last sweep of a binary32 cycle).
template <class T, bool kStream>
__global__ void __launch_bounds__(kBlock) AMG_EIGHT_WAVES k_sweep(const int *skip, int n, SellRef S,
                                                  ValRef<T> vref,
                                                  const T *__restrict__ rhs,
                                                  const T *__restrict__ x, T *__restrict__ xn,
                                                  double *__restrict__ xw) {
  AMG_SKIP_IF_DONE();
  __shared__ T sdict[kDictMax * (kBlock / kWave)];
  const ValDev<T> val = stage_dict(vref, sdict);
  val.publish();   // before any lane leaves
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r >= n) return;
  T s, m;
  sell_row<T, kStream>(S, val, x, r, s, m);
  const T di = T(1) / m;
  const T v = x[r] + di * (rhs[r] - s);
  if (xw) xw[r] = static_cast<double>(v);
  else xn[r] = v;
}

// Rows r0 and r0 + 256 of a 512-row workgroup (two slices per wavefront),
// for coded levels: out(r, sum, l1) for each row below n.
template <class T, bool kStream, class G, class F>
__device__ __forceinline__ void rows2(const SellRef &S, const ValDev<T> &V, G x, int n, int r0, F out) {
  const int r1 = r0 + kBlock;
  const int sa = __builtin_amdgcn_readfirstlane(r0 >> 6), sb = sa + kBlock / 64;
  const int nsl = (n + 63) >> 6;
  if (sa >= nsl) return;   // whole wavefront
  T s0, m0, s1, m1;
  if (sb < nsl && fold2_short<T, kStream>(S, V, x, sa, sb, r0 & 63, s0, m0, s1, m1)) {
    if (r0 < n) out(r0, s0, m0);
    if (r1 < n) out(r1, s1, m1);
    return;
  }
  V.publish();   // every lane still active
  if (r0 < n) {
    sell_row_g<T, kStream>(S, V, x, r0, s0, m0);
    out(r0, s0, m0);
  }
  if (sb < nsl && r1 < n) {
    sell_row_g<T, kStream>(S, V, x, r1, s1, m1);
    out(r1, s1, m1);
  }
}

// The sweep and the scaled residual, two slices per wavefront.
template <class T, bool kStream>
__global__ void __launch_bounds__(kBlock) AMG_EIGHT_WAVES k_sweep2(const int *skip, int n, SellRef S,
                                                   ValRef<T> vref,
                                                   const T *__restrict__ rhs,
                                                   const T *__restrict__ x, T *__restrict__ xn,
                                                   double *__restrict__ xw) {
  AMG_SKIP_IF_DONE();
  __shared__ T sdict[kDictMax * (kBlock / kWave)];
  const ValDev<T> val = stage_dict(vref, sdict);
  const int r0 = xcd_block(blockIdx.x, gridDim.x) * (2 * kBlock) + threadIdx.x;
  rows2<T, kStream>(S, val, Plain<T>{x}, n, r0, [&](int r, T sum, T l1) {
    const T di = T(1) / l1;
    const T v = x[r] + di * (rhs[r] - sum);
    if (xw) xw[r] = static_cast<double>(v);
    else xn[r] = v;
  });
}

template <class T, bool kStream>
__global__ void __launch_bounds__(kBlock) AMG_EIGHT_WAVES k_resid_scaled2(const int *skip, int n, SellRef S,
                                                          ValRef<T> vref, PVals<T> pval,
                                                          const T *__restrict__ rhs,
                                                          const T *__restrict__ x,
                                                          T *__restrict__ t) {
  AMG_SKIP_IF_DONE();
  __shared__ T sdict[kDictMax * (kBlock / kWave)];
  const ValDev<T> val = stage_dict(vref, sdict);
  const int r0 = xcd_block(blockIdx.x, gridDim.x) * (2 * kBlock) + threadIdx.x;
  rows2<T, kStream>(S, val, Plain<T>{x}, n, r0, [&](int r, T sum, T) { t[r] = pval(r) * (rhs[r] - sum); });
}

// Read in place of a null `skip`.
__device__ const int kNeverDone = 0;

// Sweep (kResid false: out = x + dinv (rhs - A x), or widened into xw) or
// scaled residual (kResid true: out = pval (rhs - A x)) on a level whose
// slices are all compact and coded with 1 to 8 slots (short_coded), two
// slices per wavefront like k_sweep2.  On the small levels a pass costs its
// memory round trips, so the loads go out in three rounds with nothing in
// between: the done flag, slice bounds, quad offsets, table entry and the
// rows' own operands; then group bases, column offsets and codes; then the
// iterate at the columns.  Same slots and fold as k_sweep2: same bits.
template <class T, bool kStream, bool kResid>
__global__ void __launch_bounds__(kBlock) AMG_EIGHT_WAVES k_short2(const int *skip, int n, SellRef S,
                                                   ValRef<T> vref, PVals<T> pval,
                                                   const T *__restrict__ rhs,
                                                   const T *__restrict__ x, T *__restrict__ out,
                                                   double *__restrict__ xw) {
  __shared__ T sdict[kDictMax * (kBlock / kWave)];
  // The kernel arguments, all read before anything else.  (The empty asm
  // statements take values as operands so that the compiler has them ready
  // at that point: loads it would otherwise issue one by one, each after the
  // previous one has returned, go out together.)
  const int *sptr = S.sptr, *qptr = S.qptr, *cbase = S.cbase;
  const int *sk = skip ? skip : &kNeverDone;
  const int nb = static_cast<int>(gridDim.x);
  asm volatile("" ::"s"(n), "s"(nb), "s"(sptr), "s"(qptr), "s"(cbase), "s"(S.cdel), "s"(vref.code),
               "s"(vref.dict), "s"(vref.ndict), "s"(pval.pval), "s"(pval.pcode), "s"(pval.pdict), "s"(rhs),
               "s"(x), "s"(out), "s"(xw), "s"(sk));
  const int r0 = xcd_block(blockIdx.x, nb) * (2 * kBlock) + threadIdx.x;
  const int r1 = r0 + kBlock;
  const int nsl = (n + 63) >> 6;
  const int sa = __builtin_amdgcn_readfirstlane(r0 >> 6);
  if (sa >= nsl) return;   // whole wavefront
  const bool two = sa + kBlock / 64 < nsl;
  const int sb = two ? sa + kBlock / 64 : sa;
  // round 1
  const int done = *sk;
  const ValDev<T> val = stage_dict(vref, sdict);
  const int ba = sptr[sa], ea = sptr[sa + 1], bb = sptr[sb], eb = sptr[sb + 1];
  const int qsa = qptr[sa], qsb = qptr[sb];
  const int ra = r0 < n ? r0 : n - 1, rb = (two && r1 < n) ? r1 : ra;
  const T oa = kResid ? pval(ra) : x[ra], ob = kResid ? pval(rb) : x[rb], ha = rhs[ra], hb = rhs[rb];
  asm volatile("" ::"s"(done), "s"(ba), "s"(ea), "s"(bb), "s"(eb), "s"(qsa), "s"(qsb));
  if (done) return;
  // round 2: the group bases (in range through the padding), then the rest
  const int wa = (ea - ba) >> 6, wb = (eb - bb) >> 6;
  const int ga = ba >> 6, gb = bb >> 6;
  int basea[8], baseb[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    basea[j] = S.cbase[ga + j];
    baseb[j] = S.cbase[gb + j];
  }
  T s0, m0, s1, m1;
  fold2_bases<T, kStream>(val, S, Plain<T>{x}, sa, sb, r0 & 63, wa, wb, qsa, qsb, basea, baseb, s0, m0,
                          s1, m1);
  auto put = [&](int r, T sum, T l1, T o, T h) {
    if constexpr (kResid) {
      out[r] = o * (h - sum);
    } else {
      const T di = T(1) / l1;
      const T v = o + di * (h - sum);
      if (xw) xw[r] = static_cast<double>(v);
      else out[r] = v;
    }
  };
  if (r0 < n) put(r0, s0, m0, oa, ha);
  if (two && r1 < n) put(r1, s1, m1, ob, hb);
}

// First post-smoothing sweep with the coarse-grid correction folded in:
// y = x + P e is formed where it is read (the value k_prolong would store)
// and xn = y + dinv (rhs - A y); y itself is never written.
template <class T, bool kStream>
__global__ void __launch_bounds__(kBlock) k_sweep_corr(const int *skip, int n, SellRef S,
                                                       ValRef<T> vref,
                                                       const T *__restrict__ rhs,
                                                       const T *__restrict__ x,
                                                       const int *__restrict__ agg,
                                                       const T *__restrict__ pval,
                                                       const T *__restrict__ e, T *__restrict__ xn) {
  AMG_SKIP_IF_DONE();
  __shared__ T sdict[kDictMax * (kBlock / kWave)];
  const ValDev<T> val = stage_dict(vref, sdict);
  val.publish();   // before any lane leaves
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r >= n) return;
  const Corrected<T> y{x, pval, agg, e};
  T s, m;
  sell_row_g<T, kStream>(S, val, y, r, s, m);
  const T di = T(1) / m;
  xn[r] = y(r) + di * (rhs[r] - s);
}

// k_sweep_corr on a short_coded level, one row per lane, in four rounds of
// loads: the done flag, slice bounds, quad offset, table entry and the
// row's own x, p, aggregate and rhs; then group bases, column offsets,
// codes and the row's e; then x, p and aggregate at the columns; then e at
// their aggregates.  Same values and fold as k_sweep_corr: same bits.
template <class T>
__global__ void __launch_bounds__(kBlock) k_short_corr(const int *skip, int n, SellRef S, ValRef<T> vref,
                                                       const T *__restrict__ rhs,
                                                       const T *__restrict__ x,
                                                       const int *__restrict__ agg,
                                                       const T *__restrict__ pval,
                                                       const T *__restrict__ e, T *__restrict__ xn) {
  __shared__ T sdict[kDictMax * (kBlock / kWave)];
  const int *sptr = S.sptr, *qptr = S.qptr, *cbase = S.cbase;
  const int *sk = skip ? skip : &kNeverDone;
  const int nb = static_cast<int>(gridDim.x);
  asm volatile("" ::"s"(n), "s"(nb), "s"(sptr), "s"(qptr), "s"(cbase), "s"(S.cdel), "s"(vref.code),
               "s"(vref.dict), "s"(vref.ndict), "s"(rhs), "s"(x), "s"(agg), "s"(pval), "s"(e), "s"(xn),
               "s"(sk));
  const int r = xcd_block(blockIdx.x, nb) * kBlock + threadIdx.x;
  const int sl = __builtin_amdgcn_readfirstlane(r >> 6);
  if (sl >= ((n + 63) >> 6)) return;   // whole wavefront
  // round 1
  const int done = *sk;
  const ValDev<T> val = stage_dict(vref, sdict);
  const int b = sptr[sl], en = sptr[sl + 1], qs = qptr[sl];
  const int rr = r < n ? r : n - 1;
  const T xr = x[rr], pr = pval[rr], hr = rhs[rr];
  const int ar = agg[rr];
  asm volatile("" ::"s"(done), "s"(b), "s"(en), "s"(qs));
  if (done) return;
  // round 2
  const int w = (en - b) >> 6, g = b >> 6, lane = r & 63;
  int base[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) base[j] = cbase[g + j];   // in range through the padding
  const T er = e[ar];
  const unsigned long long *cd = reinterpret_cast<const unsigned long long *>(S.cdel);
  const unsigned *cc = reinterpret_cast<const unsigned *>(val.code);
  const int64_t qa = static_cast<int64_t>(qs) * 64 + lane;
  const int t2 = w > 4 ? 64 : 0;
  const unsigned long long d0 = cd[qa], d1 = cd[qa + t2];
  const unsigned k0 = cc[qa], k1 = cc[qa + t2];
  // round 3
  int c[8], ac[8];
  T xc[8], pc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const unsigned long long d = j < 4 ? d0 : d1;
    c[j] = j < w ? base[j] + static_cast<int>((d >> (16 * (j & 3))) & 0xffffu) : sl * 64;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    xc[j] = x[c[j]];
    pc[j] = pval[c[j]];
    ac[j] = agg[c[j]];
  }
  // round 4
  T ec[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) ec[j] = e[ac[j]];
  val.publish();
  T acc = T(0), m = T(0);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const unsigned kk = j < 4 ? k0 : k1;
    const T a = val.mine[(kk >> (8 * (j & 3))) & 0xffu];
    if (j < w) {
      acc = acc + a * (xc[j] + pc[j] * ec[j]);
      m = m + fabs(a);
    }
  }
  if (r < n) {
    const T di = T(1) / m;
    xn[r] = (xr + pr * er) + di * (hr - acc);
  }
}

// First sweep from x = 0: x = dinv * r.
template <class T>
__global__ void __launch_bounds__(kBlock) k_sweep_first(const int *skip, int n,
                                                        const T *__restrict__ dinv,
                                                        const T *__restrict__ rhs,
                                                        T *__restrict__ x) {
  AMG_SKIP_IF_DONE();
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r < n) x[r] = dinv[r] * rhs[r];
}

// Restriction, pass 1 (row parallel): t_i = p_i (r_i - (A x)_i).
template <class T, bool kStream>
__global__ void __launch_bounds__(kBlock) AMG_EIGHT_WAVES k_resid_scaled(const int *skip, int n, SellRef S,
                                                         ValRef<T> vref,
                                                         const T *__restrict__ pval,
                                                         const T *__restrict__ rhs,
                                                         const T *__restrict__ x,
                                                         T *__restrict__ t) {
  AMG_SKIP_IF_DONE();
  __shared__ T sdict[kDictMax * (kBlock / kWave)];
  const ValDev<T> val = stage_dict(vref, sdict);
  val.publish();   // before any lane leaves
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r >= n) return;
  T s, m;
  sell_row<T, kStream>(S, val, x, r, s, m);
  t[r] = pval[r] * (rhs[r] - s);
}

// Restriction, pass 2 (aggregate parallel): r_c[I] = sum of t over the
// members of I in ascending order.  When the coarse level starts with a
// smoothing sweep its first iterate x_c = dinv_c r_c is written as well.
template <class T>
__global__ void __launch_bounds__(kBlock) k_agg_sum(const int *skip, int nc,
                                                    const int *__restrict__ mptr,
                                                    const int *__restrict__ mem,
                                                    const T *__restrict__ t, T *__restrict__ rc,
                                                    const T *__restrict__ dinvc,
                                                    T *__restrict__ xc) {
  AMG_SKIP_IF_DONE();
  const int I = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (I >= nc) return;
  T acc = T(0);
  for (int q = mptr[I]; q < mptr[I + 1]; ++q) acc = acc + t[mem[q]];
  rc[I] = acc;
  if (xc) xc[I] = dinvc[I] * acc;
}

// Restriction in one pass (small levels, where the two passes above are
// bound by launch latency): G lanes per aggregate; lane q forms the scaled
// residual t = p_i (r_i - (A x)_i) of member q (ascending), its row folded
// in CSR order (the SELL slot order; padding slots add zeros), and the first
// lane of the group adds the members' values in order; members beyond G are
// folded by that lane itself.  Same bits as k_resid_scaled + k_agg_sum.
template <class T, int G, bool kShort = false>
__global__ void __launch_bounds__(kBlock) k_resid_agg(const int *skip, int nc,
                                                      const int *__restrict__ mptr,
                                                      const int *__restrict__ mem,
                                                      const int *__restrict__ rp,
                                                      const int *__restrict__ ci,
                                                      const double *__restrict__ v,
                                                      const T *__restrict__ pval,
                                                      const T *__restrict__ rhs,
                                                      const T *__restrict__ x, T *__restrict__ rc,
                                                      const T *__restrict__ dinvc, T *__restrict__ xc) {
  // kShort (rows of at most 8 entries): the kernel arguments, the done
  // flag, the aggregate's bounds and its diagonal go out together, and a
  // row's entries in one batch (see k_short2 for the empty asm statements)
  const int *sk = skip ? skip : &kNeverDone;
  const int nb = static_cast<int>(gridDim.x);
  if constexpr (kShort) {
    asm volatile("" ::"s"(nc), "s"(nb), "s"(mptr), "s"(mem), "s"(rp), "s"(ci), "s"(v), "s"(pval), "s"(rhs),
                 "s"(x), "s"(rc), "s"(dinvc), "s"(xc), "s"(sk));
  } else {
    AMG_SKIP_IF_DONE();
  }
  const int e = xcd_block(blockIdx.x, nb) * kBlock + threadIdx.x;
  const int I = e / G, q = e % G;
  const bool live = I < nc;
  int q0 = 0, cnt = 0;
  T dI = T(0);
  if (live) {
    q0 = mptr[I];
    cnt = mptr[I + 1] - q0;
    if (kShort && xc) dI = dinvc[I];
  }
  if constexpr (kShort) {
    const int done = *sk;
    asm volatile("" ::"s"(done), "v"(q0), "v"(cnt));
    if (done) return;
  }
  constexpr int KB = kShort ? 8 : 4;
  auto scaled = [&](int i) {   // entries taken KB at a time, all loads of a batch in flight
    const T pi = pval[i], hi = rhs[i];
    T acc = T(0);
    int k = rp[i];
    const int k1 = rp[i + 1];
    for (; k < k1; k += KB) {
      int c[KB];
      T a[KB], xv[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u)
        if (k + u < k1) {
          c[u] = ci[k + u];
          a[u] = static_cast<T>(v[k + u]);
        }
#pragma unroll
      for (int u = 0; u < KB; ++u)
        if (k + u < k1) xv[u] = x[c[u]];
#pragma unroll
      for (int u = 0; u < KB; ++u)
        if (k + u < k1) acc = acc + a[u] * xv[u];
    }
    return pi * (hi - acc);
  };
  T t = T(0);
  if (q < cnt) t = scaled(mem[q0 + q]);
  const int lead = (threadIdx.x & (kWave - 1)) - q;
  T acc = T(0);
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const T tj = __shfl(t, lead + j, kWave);
    if (j < cnt) acc = acc + tj;
  }
  if (!live || q != 0) return;
  for (int j = G; j < cnt; ++j) acc = acc + scaled(mem[q0 + j]);
  rc[I] = acc;
  if (xc) xc[I] = (kShort ? dI : dinvc[I]) * acc;
}

// x_i += p_i * e[agg_i]
template <class T>
__global__ void __launch_bounds__(kBlock) k_prolong(const int *skip, int n,
                                                    const int *__restrict__ agg, PVals<T> pval,
                                                    const T *__restrict__ e, T *__restrict__ x) {
  AMG_SKIP_IF_DONE();
  const int r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r < n) x[r] = x[r] + pval(r) * e[agg[r]];
}

template <class T>
__global__ void k_zero(const int *skip, int n, T *x) {
  AMG_SKIP_IF_DONE();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) x[r] = T(0);
}

// Mixed precision entry: rf = (float) r and, if the fine level starts with a
// sweep, its first iterate x = dinv * rf.
__global__ void __launch_bounds__(kBlock) k_d2f_first(const int *skip, int n,
                                                      const double *__restrict__ r,
                                                      const float *__restrict__ dinv,
                                                      float *__restrict__ rf,
                                                      float *__restrict__ x) {
  AMG_SKIP_IF_DONE();
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const float b = static_cast<float>(r[i]);
  rf[i] = b;
  if (x) x[i] = dinv[i] * b;
}

__global__ void k_f2d(const int *skip, int n, const float *__restrict__ a, double *__restrict__ b) {
  AMG_SKIP_IF_DONE();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = static_cast<double>(a[r]);
}

__global__ void k_d2f(const int *skip, int n, const double *__restrict__ a, float *__restrict__ b) {
  AMG_SKIP_IF_DONE();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = static_cast<float>(a[r]);
}

// Mixed precision, coarsest level solved by sweeps: the binary32 right-hand
// side widened to binary64 (rd) and the first binary64 iterate x = dinv * rd.
__global__ void __launch_bounds__(kBlock) k_f2d_first(const int *skip, int n,
                                                      const float *__restrict__ rf,
                                                      const double *__restrict__ dinv,
                                                      double *__restrict__ rd,
                                                      double *__restrict__ x) {
  AMG_SKIP_IF_DONE();
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const double b = static_cast<double>(rf[i]);
  rd[i] = b;
  x[i] = dinv[i] * b;
}

// ------------------------------------------------------ coarse-tail kernel
// Levels [kt, nl) of the V-cycle in ONE workgroup, thread i owning row i
// (and aggregate i) of every level.  All vectors of these levels live in
// LDS (r, two iterates, scaled residual: 4 n_j entries per level); a
// thread keeps its matrix row in registers while it works on a level
// (slots beyond W are re-read from memory), so a smoothing sweep costs LDS
// gathers and one workgroup barrier.  Every fold is the one of the
// multi-workgroup kernels: slots in order for rows and l1 norms, members in
// ascending order for the restriction.
// Coarsest level: z = A^-1 r with the column-major inverse, row i folded
// over j ascending, in binary64 (also for the binary32 cycle); or l1-Jacobi
// sweeps.
template <class T, int W>
struct TailRow {
  T v[W];
  int c[W];
  int w;             // slots of the row's slice (k >= W read through cp / vp)
  const int *cp;
  const T *vp;
  T dinv;            // 1 / sum_k |a_k|, the fold of the stored diagonal
};

template <class T, int W>
__device__ __forceinline__ void tail_load(const TailDesc<T> &L, int r, TailRow<T, W> &R) {
  const int s = r >> 6, lane = r & 63;
  const int b = L.sptr[s];
  R.w = (L.sptr[s + 1] - b) >> 6;
  R.cp = L.col + b + lane;
  R.vp = L.val + b + lane;
#pragma unroll
  for (int k = 0; k < W; ++k)
    if (k < R.w) {
      R.c[k] = R.cp[k * 64];
      R.v[k] = R.vp[k * 64];
    }
  T m = T(0);
#pragma unroll
  for (int k = 0; k < W; ++k)
    if (k < R.w) m = m + fabs(R.v[k]);
  for (int k = W; k < R.w; ++k) m = m + fabs(R.vp[k * 64]);
  R.dinv = T(1) / m;
}

template <class T, int W>
__device__ __forceinline__ T tail_dot(const TailRow<T, W> &R, const T *X) {
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < W; ++k)
    if (k < R.w) acc = acc + R.v[k] * X[R.c[k]];
  for (int k = W; k < R.w; ++k) acc = acc + R.vp[k * 64] * X[R.cp[k * 64]];
  return acc;
}

// The direct coarsest solve of the tail kernels, X = A^-1 rhs with the
// explicit inverse (binary64): X_i = sum over c ascending of Ainv[c n + i]
// rhs_c.  The workgroup forms the products of K columns at a time (one
// coalesced load per thread) into LDS, then thread i adds its row's
// products in column order: the same products and the same order of sums
// as a row-by-row loop, with one memory round trip per K columns instead of
// a chain of them.  n <= the workgroup size; called by the whole workgroup.
constexpr int kTailGemv = 4096;   // LDS doubles for the staged products
static_assert(kDenseMax <= kTailThreads, "one thread per row of the dense coarsest level");

template <class T>
__device__ __forceinline__ void tail_dense_solve(int n, const double *__restrict__ Ainv, const T *rhs, T *X,
                                                 double *P) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int K = max(1, min(n, kTailGemv / n));
  double acc = 0.0;
  for (int c0 = 0; c0 < n; c0 += K) {
    const int kc = min(K, n - c0);
    for (int e = t; e < kc * n; e += nt) {
      const int cc = e / n, i = e - cc * n;
      P[e] = Ainv[static_cast<int64_t>(c0 + cc) * n + i] * static_cast<double>(rhs[c0 + cc]);
    }
    __syncthreads();
    if (t < n)
      for (int cc = 0; cc < kc; ++cc) acc = acc + P[cc * n + t];
    __syncthreads();
  }
  if (t < n) X[t] = static_cast<T>(acc);
}

template <class T, int W>
__global__ void __launch_bounds__(kTailThreads) k_vcycle_tail(
    const int *skip, int m, const TailDesc<T> *__restrict__ D, const double *__restrict__ Ainv,
    int dense, int pre, int post, int csw, const T *__restrict__ top_rhs, T *__restrict__ top_out) {
  AMG_SKIP_IF_DONE();
  __shared__ T lds[kTailLds];
  __shared__ double gemv[kTailGemv];
  const int t = threadIdx.x, nt = blockDim.x;
  // level j: R = lds + off, X0 = R + n, X1 = R + 2n, Tt = R + 3n; bit j of
  // `sel` says which iterate holds the level's current x (uniform)
  unsigned long long sel = 0;
  {
    const TailDesc<T> L = D[0];
    for (int i = t; i < L.n; i += nt) lds[L.lds + i] = top_rhs[i];
  }
  __syncthreads();
  // ---- descent
  for (int j = 0; j < m - 1; ++j) {
    const TailDesc<T> L = D[j];
    const TailDesc<T> C = D[j + 1];
    const int n = L.n;
    const T *rhs = lds + L.lds;
    T *X = lds + L.lds + n, *Y = lds + L.lds + 2 * n, *Tt = lds + L.lds + 3 * n;
    TailRow<T, W> R;
    T pv = T(0);
    // members of aggregate t (up to 8 kept in registers), read ahead of use
    int mb = 0, mc = 0, mm[8];
    if (t < L.nc) {
      mb = L.mptr[t];
      mc = L.mptr[t + 1] - mb;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < mc) mm[k] = L.mem[mb + k];
    }
    if (t < n) {
      tail_load<T, W>(L, t, R);
      pv = L.pval[t];
      X[t] = (pre > 0) ? R.dinv * rhs[t] : T(0);
    }
    __syncthreads();
    for (int q = 1; q < pre; ++q) {
      if (t < n) Y[t] = X[t] + R.dinv * (rhs[t] - tail_dot<T, W>(R, X));
      __syncthreads();
      T *tmp = X; X = Y; Y = tmp;
    }
    if (t < n) Tt[t] = pv * (rhs[t] - tail_dot<T, W>(R, X));
    if (X != lds + L.lds + n) sel |= 1ull << j;
    __syncthreads();
    if (t < L.nc) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < mc) acc = acc + Tt[mm[k]];
      for (int k = 8; k < mc; ++k) acc = acc + Tt[L.mem[mb + k]];
      lds[C.lds + t] = acc;
    }
    __syncthreads();
  }
  // ---- coarsest level (result in its X0 or X1, recorded in sel)
  {
    const int j = m - 1;
    const TailDesc<T> L = D[j];
    const int n = L.n;
    const T *rhs = lds + L.lds;
    T *X = lds + L.lds + n, *Y = lds + L.lds + 2 * n;
    if (dense) {
      tail_dense_solve<T>(n, Ainv, rhs, X, gemv);
    } else {
      TailRow<T, W> R;
      if (t < n) {
        tail_load<T, W>(L, t, R);
        X[t] = R.dinv * rhs[t];
      }
      __syncthreads();
      for (int q = 1; q < csw; ++q) {
        if (t < n) Y[t] = X[t] + R.dinv * (rhs[t] - tail_dot<T, W>(R, X));
        __syncthreads();
        T *tmp = X; X = Y; Y = tmp;
      }
    }
    if (X != lds + L.lds + n) sel |= 1ull << j;
    __syncthreads();
  }
  // ---- ascent: x += P e, then the post-smoothing sweeps
  for (int j = m - 2; j >= 0; --j) {
    const TailDesc<T> L = D[j];
    const TailDesc<T> C = D[j + 1];
    const int n = L.n;
    const T *rhs = lds + L.lds;
    T *X = lds + L.lds + ((sel >> j) & 1 ? 2 * n : n);
    T *Y = lds + L.lds + ((sel >> j) & 1 ? n : 2 * n);
    const T *e = lds + C.lds + ((sel >> (j + 1)) & 1 ? 2 * C.n : C.n);
    TailRow<T, W> R;
    if (t < n) {
      X[t] = X[t] + L.pval[t] * e[L.agg[t]];
      if (post > 0) tail_load<T, W>(L, t, R);
    }
    __syncthreads();
    for (int q = 0; q < post; ++q) {
      if (t < n) Y[t] = X[t] + R.dinv * (rhs[t] - tail_dot<T, W>(R, X));
      __syncthreads();
      T *tmp = X; X = Y; Y = tmp;
    }
    if (X != lds + L.lds + n) sel |= 1ull << j;
    else sel &= ~(1ull << j);
  }
  {
    const TailDesc<T> L = D[0];
    const T *X = lds + L.lds + ((sel & 1) ? 2 * L.n : L.n);
    for (int i = t; i < L.n; i += nt) top_out[i] = X[i];
  }
}

// Coarse tail of the general cycle (binary64, l1-Jacobi smoothing on every
// level, direct or l1-Jacobi coarsest solve) for V-, H- and W-cycles: the
// levels from the tail's first on, in one workgroup.  Level j of the tail
// (level k0 + j of the hierarchy) makes g_j coarse-grid corrections per
// visit: e = C(r_c), then e += C(r_c - A_c e) (W: g = 2; H: g = 2 on odd
// levels; V: g = 1).  The recursion runs as a loop over (level, direction)
// with the per-level state in bit masks (uniform over the workgroup).  Five
// LDS vectors per level: right-hand side, two iterates, scaled residual, and
// E, the sum of the corrections this level's cycles return to the level
// above.  Same operations and fold orders as the kernel-by-kernel cycle.
template <int W>
__global__ void __launch_bounds__(kTailThreads) k_cycle_tail_g(
    const int *skip, int m, int k0, int cycle, const TailDesc<double> *__restrict__ D,
    const double *__restrict__ Ainv, int dense, int pre, int post, int csw,
    const double *__restrict__ top_rhs, double *__restrict__ top_out) {
  AMG_SKIP_IF_DONE();
  __shared__ double lds[kTailLds];
  __shared__ double gemv[kTailGemv];
  const int t = threadIdx.x, nt = blockDim.x;
  auto corrections = [&](int j) {
    const int k = k0 + j;
    return cycle == AMG_CYCLE_W ? 2 : (cycle == AMG_CYCLE_H && k % 2 == 1 ? 2 : 1);
  };
  unsigned long long sel = 0;     // bit j: level j's current iterate is its second one
  unsigned long long more = 0;    // bit j: level j still owes a second correction
  unsigned long long first = 0;   // bit j: level j has not received a correction yet
  auto iterate = [&](const TailDesc<double> &L, int j) {
    return lds + L.lds + (((sel >> j) & 1) ? 2 : 1) * L.n;
  };
  {
    const TailDesc<double> L = D[0];
    for (int i = t; i < L.n; i += nt) lds[L.lds + i] = top_rhs[i];
  }
  __syncthreads();
  int j = 0;
  bool down = true;
  for (;;) {
    const TailDesc<double> L = D[j];
    const int n = L.n;
    double *rhs = lds + L.lds;
    if (down && j == m - 1) {
      // ---- coarsest level, from zero
      double *X = rhs + n, *Y = rhs + 2 * n;
      if (dense) {
        tail_dense_solve<double>(n, Ainv, rhs, X, gemv);
      } else {
        TailRow<double, W> R;
        if (t < n) {
          tail_load<double, W>(L, t, R);
          X[t] = R.dinv * rhs[t];
        }
        __syncthreads();
        for (int q = 1; q < csw; ++q) {
          if (t < n) Y[t] = X[t] + R.dinv * (rhs[t] - tail_dot<double, W>(R, X));
          __syncthreads();
          double *tmp = X; X = Y; Y = tmp;
        }
      }
      if (X != rhs + n) sel |= 1ull << j;
      else sel &= ~(1ull << j);
      __syncthreads();
      if (j == 0) break;
      --j;
      down = false;
      continue;
    }
    if (down) {
      // ---- pre-smoothing from zero, scaled residual, restriction
      const TailDesc<double> C = D[j + 1];
      double *X = rhs + n, *Y = rhs + 2 * n, *Tt = rhs + 3 * n;
      TailRow<double, W> R;
      double pv = 0.0;
      int mb = 0, mc = 0, mm[8];
      if (t < L.nc) {
        mb = L.mptr[t];
        mc = L.mptr[t + 1] - mb;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k < mc) mm[k] = L.mem[mb + k];
      }
      if (t < n) {
        tail_load<double, W>(L, t, R);
        pv = L.pval[t];
        X[t] = (pre > 0) ? R.dinv * rhs[t] : 0.0;
      }
      __syncthreads();
      for (int q = 1; q < pre; ++q) {
        if (t < n) Y[t] = X[t] + R.dinv * (rhs[t] - tail_dot<double, W>(R, X));
        __syncthreads();
        double *tmp = X; X = Y; Y = tmp;
      }
      if (t < n) Tt[t] = pv * (rhs[t] - tail_dot<double, W>(R, X));
      if (X != rhs + n) sel |= 1ull << j;
      else sel &= ~(1ull << j);
      __syncthreads();
      if (t < L.nc) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k < mc) acc = acc + Tt[mm[k]];
        for (int k = 8; k < mc; ++k) acc = acc + Tt[L.mem[mb + k]];
        lds[C.lds + t] = acc;
      }
      __syncthreads();
      first |= 1ull << j;
      if (corrections(j) > 1) more |= 1ull << j;
      else more &= ~(1ull << j);
      ++j;
      continue;
    }
    // ---- up: level j receives the result of a cycle on level j + 1
    const TailDesc<double> C = D[j + 1];
    const double *e_in = iterate(C, j + 1);
    double *Ebuf = lds + C.lds + 4 * C.n;
    const bool is_first = (first >> j) & 1, owes = (more >> j) & 1;
    const double *E = e_in;
    if (!is_first || owes) {
      for (int i = t; i < C.n; i += nt) Ebuf[i] = is_first ? e_in[i] : Ebuf[i] + e_in[i];
      __syncthreads();
      E = Ebuf;
    }
    first &= ~(1ull << j);
    if (owes) {
      // r_c <- r_c - A_c e (each row reads and writes only its own entry of r_c)
      more &= ~(1ull << j);
      double *rc = lds + C.lds;
      if (t < C.n) {
        TailRow<double, W> Rc;
        tail_load<double, W>(C, t, Rc);
        rc[t] = rc[t] - tail_dot<double, W>(Rc, E);
      }
      __syncthreads();
      ++j;
      down = true;
      continue;
    }
    // ---- x += P e, then the post-smoothing sweeps
    {
      double *X = iterate(L, j);
      double *Y = (X == rhs + n) ? rhs + 2 * n : rhs + n;
      TailRow<double, W> R;
      if (t < n) {
        X[t] = X[t] + L.pval[t] * E[L.agg[t]];
        if (post > 0) tail_load<double, W>(L, t, R);
      }
      __syncthreads();
      for (int q = 0; q < post; ++q) {
        if (t < n) Y[t] = X[t] + R.dinv * (rhs[t] - tail_dot<double, W>(R, X));
        __syncthreads();
        double *tmp = X; X = Y; Y = tmp;
      }
      if (X != rhs + n) sel |= 1ull << j;
      else sel &= ~(1ull << j);
    }
    if (j == 0) break;
    --j;
  }
  {
    const TailDesc<double> L = D[0];
    const double *X = iterate(L, 0);
    for (int i = t; i < L.n; i += nt) top_out[i] = X[i];
  }
}

// ----------------------------------------------------------- PCG kernels
constexpr int kFinish = 1024;   // threads of the one-workgroup finishing kernels
constexpr int kRowsDot = 2;     // rows per thread in the SpMV + dots kernels
constexpr int kRowsUpd = 4;     // elements per thread in the vector update

// Deterministic workgroup sum (fixed butterfly in each wave, waves in order).
template <int NT>
__device__ __forceinline__ double group_sum(double v, double *red) {
  v = wave_sum(v);
  const int wid = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[wid] = v;
  __syncthreads();
  double t = red[0];
  for (int q = 1; q < NT / kWave; ++q) t = t + red[q];
  __syncthreads();
  return t;
}

// Fold part[q*3 + o], q = 0..np-1, for o < NQ: each thread folds its
// indices q = tid, tid + 1024, ... in order (up to 8192 partials: all loads
// of a thread in flight at once; beyond, four at a time), then the
// workgroup sum combines the threads in a fixed order.
template <int NQ>
__device__ __forceinline__ void fold_parts(const double *__restrict__ part, int np, double *red,
                                           double *out) {
  double acc[NQ];
#pragma unroll
  for (int o = 0; o < NQ; ++o) acc[o] = 0.0;
  int q = threadIdx.x;
  if (np <= 8 * kFinish) {
    double v[8][NQ];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int o = 0; o < NQ; ++o)
        if (q + u * kFinish < np) v[u][o] = part[(q + u * kFinish) * 3 + o];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q + u * kFinish < np)
#pragma unroll
        for (int o = 0; o < NQ; ++o) acc[o] = acc[o] + v[u][o];
    q = np;
  }
  for (; q + 3 * kFinish < np; q += 4 * kFinish) {
    double v[4][NQ];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int o = 0; o < NQ; ++o) v[u][o] = part[(q + u * kFinish) * 3 + o];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int o = 0; o < NQ; ++o) acc[o] = acc[o] + v[u][o];
  }
  for (; q < np; q += kFinish)
#pragma unroll
    for (int o = 0; o < NQ; ++o) acc[o] = acc[o] + part[q * 3 + o];
#pragma unroll
  for (int o = 0; o < NQ; ++o) out[o] = group_sum<kFinish>(acc[o], red);
}

// Optional outputs of the kernels that produce the PCG residual r: the first
// smoothing iterate of the next V-cycle (x = dinv * r), or for the binary32
// cycle rf = (float) r and x = dinv_f * rf.  Null pointers disable them.
struct FirstOut {
  const double *dinv;
  double *x;
  const float *dinvf;
  float *rf;
  float *xf;
};

__device__ __forceinline__ void first_out(const FirstOut &fo, int i, double ri) {
  if (fo.x) fo.x[i] = fo.dinv[i] * ri;
  if (fo.rf) {
    const float b = static_cast<float>(ri);
    fo.rf[i] = b;
    if (fo.xf) fo.xf[i] = fo.dinvf[i] * b;
  }
}

// r = b - A u, partial ||r||^2 per workgroup (kRowsDot rows per thread).
template <bool kStream>
// r = b - A x0 with x0 the caller's initial guess; the iterate u = x0 and
// the recurrences' d = q = 0 are written here too (no separate passes).
__global__ void __launch_bounds__(kBlock) k_pcg_init(int n, SellRef S,
                                                     ValRef<double> vref,
                                                     const double *__restrict__ b,
                                                     const double *__restrict__ x0,
                                                     double *__restrict__ u, double *__restrict__ d,
                                                     double *__restrict__ q, double *__restrict__ r,
                                                     double *__restrict__ part, FirstOut fo) {
  __shared__ double red[kBlock / kWave];
  __shared__ double sdict[kDictMax * (kBlock / kWave)];
  const ValDev<double> val = stage_dict(vref, sdict);
  val.publish();   // before any lane leaves
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  double rr = 0.0;
#pragma unroll
  for (int h = 0; h < kRowsDot; ++h) {
    const int row = (lb * kRowsDot + h) * kBlock + threadIdx.x;
    if (row < n) {
      double s, m;
      sell_row<double, kStream>(S, val, x0, row, s, m);
      const double ri = b[row] - s;
      r[row] = ri;
      u[row] = x0[row];
      d[row] = 0.0;
      q[row] = 0.0;
      first_out(fo, row, ri);
      rr = rr + ri * ri;
    }
  }
  rr = group_sum<kBlock>(rr, red);
  if (threadIdx.x == 0) part[lb * 3] = rr;
}

__global__ void __launch_bounds__(kFinish) k_pcg_init_finish(int nb, const double *part,
                                                             Scalars *sc, double rtol, int maxit) {
  __shared__ double red[kFinish / kWave];
  double tot;
  fold_parts<1>(part, nb, red, &tot);
  if (threadIdx.x == 0) {
    const double nr0 = sqrt(tot);
    sc->nr0 = nr0;
    sc->rr = tot;
    sc->thr = rtol * nr0;
    sc->rho = 1.0;
    sc->c = 0.0;
    sc->a = 0.0;
    sc->it = 0;
    sc->maxit = maxit;
    sc->conv = (nr0 == 0.0) ? 1 : 0;
    sc->status = isfinite(nr0) ? 0 : AMG_ERR_NONFINITE;
    sc->done = (nr0 == 0.0 || !isfinite(nr0)) ? 1 : 0;
  }
}

// v = A w and partial dots alpha = w.r, beta = w.v, gamma = w.q.
template <bool kStream>
__global__ void __launch_bounds__(kBlock) AMG_EIGHT_WAVES k_pcg_spmv_dots(
    const int *skip, int n, SellRef S, ValRef<double> vref, const double *__restrict__ w,
    const double *__restrict__ r,
    const double *__restrict__ q, double *__restrict__ v, double *__restrict__ part) {
  AMG_SKIP_IF_DONE();
  __shared__ double red[kBlock / kWave];
  __shared__ double sdict[kDictMax * (kBlock / kWave)];
  const ValDev<double> val = stage_dict(vref, sdict);
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  double al = 0.0, be = 0.0, ga = 0.0;
  static_assert(kRowsDot == 2, "rows r and r + kBlock of the workgroup's 2 kBlock rows");
  rows2<double, kStream>(S, val, Plain<double>{w}, n, lb * kRowsDot * kBlock + threadIdx.x,
                         [&](int row, double s, double) {
                           v[row] = s;
                           const double wi = w[row];
                           al = al + wi * r[row];
                           be = be + wi * s;
                           ga = ga + wi * q[row];
                         });
  al = group_sum<kBlock>(al, red);
  be = group_sum<kBlock>(be, red);
  ga = group_sum<kBlock>(ga, red);
  if (threadIdx.x == 0) {
    part[lb * 3 + 0] = al;
    part[lb * 3 + 1] = be;
    part[lb * 3 + 2] = ga;
  }
}

// rho_i = beta - gamma^2 / rho_{i-1}; c = gamma / rho_{i-1}; a = alpha / rho_i (Alg. 1).
__global__ void __launch_bounds__(kFinish) k_pcg_dots_finish(const int *skip, int nb,
                                                             const double *part, Scalars *sc) {
  AMG_SKIP_IF_DONE();
  __shared__ double red[kFinish / kWave];
  const double rho_prev = sc->rho;   // read with the partials
  double t[3];
  fold_parts<3>(part, nb, red, t);
  if (threadIdx.x == 0) {
    const double A = t[0], B = t[1], G = t[2];
    const double rho = B - (G * G) / rho_prev;
    sc->alpha = A;
    sc->beta = B;
    sc->gamma = G;
    sc->it = sc->it + 1;
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
  }
}

// d = w - c d; u = u + a d; q = v - c q; r = r - a q; partial ||r||^2.
__global__ void __launch_bounds__(kBlock) k_pcg_update(const int *skip, int n,
                                                       const double *__restrict__ w,
                                                       const double *__restrict__ v,
                                                       double *__restrict__ d,
                                                       double *__restrict__ u,
                                                       double *__restrict__ q,
                                                       double *__restrict__ r,
                                                       const Scalars *__restrict__ sc,
                                                       double *__restrict__ part, FirstOut fo) {
  AMG_SKIP_IF_DONE();
  __shared__ double red[kBlock / kWave];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const double c = sc->c, a = sc->a;
  double rr = 0.0;
#pragma unroll
  for (int h = 0; h < kRowsUpd; ++h) {
    const int i = (lb * kRowsUpd + h) * kBlock + threadIdx.x;
    if (i < n) {
      // w, v, d, u, q are not read again before the next update: non-temporal
      // accesses keep them from displacing the fine matrix and r, which the
      // V-cycle reads next, from the last-level cache
      const double di = ld_stream(w + i) - c * ld_stream(d + i);
      __builtin_nontemporal_store(di, d + i);
      __builtin_nontemporal_store(ld_stream(u + i) + a * di, u + i);
      const double qi = ld_stream(v + i) - c * ld_stream(q + i);
      __builtin_nontemporal_store(qi, q + i);
      const double ri = r[i] - a * qi;
      r[i] = ri;
      first_out(fo, i, ri);
      rr = rr + ri * ri;
    }
  }
  rr = group_sum<kBlock>(rr, red);
  if (threadIdx.x == 0) part[lb * 3] = rr;
}

// ||r|| <= rtol ||r_0|| ends the iteration (Sec. 5); so do a non-finite norm
// and the iteration limit.  The state is then copied to host-coherent pinned
// memory (also when the iteration was skipped), which the host polls.
__global__ void __launch_bounds__(kFinish) k_pcg_norm_finish(const int *skip, int nb,
                                                             const double *part, Scalars *sc,
                                                             Scalars *host) {
  __shared__ double red[kFinish / kWave];
  const bool live = !(*skip);
  const double thr = sc->thr;   // read with the partials
  const int it = sc->it, maxit = sc->maxit;
  double tot = 0.0;
  if (live) fold_parts<1>(part, nb, red, &tot);
  if (threadIdx.x == 0) {
    if (live) {
      const double nr = sqrt(tot);
      sc->rr = tot;
      if (nr <= thr) {
        sc->conv = 1;
        sc->done = 1;
      } else if (!isfinite(nr)) {
        sc->status = AMG_ERR_NONFINITE;
        sc->done = 1;
      } else if (it >= maxit) {
        sc->done = 1;
      }
    }
    *host = *sc;
  }
}

// ------------------------------------------------------------ V-cycle
template <class T> const T *dinv_of(const Level &L);
template <> const double *dinv_of<double>(const Level &L) { return L.dinv.p; }
template <> const float *dinv_of<float>(const Level &L) { return L.dinvf.p; }
template <class T> const T *pval_of(const Level &L);
template <> const double *pval_of<double>(const Level &L) { return L.pval.p; }
template <> const float *pval_of<float>(const Level &L) { return L.pvalf.p; }
// P values for the kernels that read them coded when the level has codes
// (binary64 cycle: 1 byte instead of 8 per row, 160^3 solve 9.05 -> 8.95 ms;
// the binary32 cycle reads pvalf, 7.26 ms against 7.33 ms with codes, where
// the table lookup's extra round trip outweighs 3 bytes per row)
template <class T> PVals<T> pvals_of(const Level &L);
template <> PVals<double> pvals_of<double>(const Level &L) {
  return PVals<double>{L.pval.p, L.npdict ? L.pcode.p : nullptr, L.pdict.p};
}
template <> PVals<float> pvals_of<float>(const Level &L) { return PVals<float>{L.pvalf.p, nullptr, nullptr}; }
template <class T> PVals<T> plain_pvals(const T *p) { return PVals<T>{p, nullptr, nullptr}; }
template <class T> T *rbuf(Level &L);
template <> double *rbuf<double>(Level &L) { return L.r.p; }
template <> float *rbuf<float>(Level &L) { return L.rf.p; }
template <class T> T *xbuf(Level &L);
template <> double *xbuf<double>(Level &L) { return L.x.p; }
template <> float *xbuf<float>(Level &L) { return L.xf.p; }
template <class T> T *tbuf(Level &L);
template <> double *tbuf<double>(Level &L) { return L.t.p; }
template <> float *tbuf<float>(Level &L) { return L.tf.p; }

template <class T> const TailDesc<T> *tail_desc(amg_hierarchy *h);
template <> const TailDesc<double> *tail_desc<double>(amg_hierarchy *h) {
  return reinterpret_cast<const TailDesc<double> *>(h->tail_desc_d.p);
}
template <> const TailDesc<float> *tail_desc<float>(amg_hierarchy *h) {
  return reinterpret_cast<const TailDesc<float> *>(h->tail_desc_f.p);
}

// Matrices at least this large are read with non-temporal loads; smaller
// ones use plain loads, so that a level's matrix can stay in the last-level
// cache (256 MB on MI355X) between the passes of one V-cycle.  (Measured at
// 160^3: the binary64 fine level, 287 MB, is faster streamed; the binary32
// copy, 172 MB, is faster read with plain loads.)
#ifndef AMG_STREAM_MIN_MB
#define AMG_STREAM_MIN_MB 200
#endif
template <class T>
bool streamed(const Level &L) {
  const double bytes = static_cast<double>(L.S.nslots) * ((L.S.ndict ? 1.0 : sizeof(T)) + 2.0);
  return bytes >= AMG_STREAM_MIN_MB * 1048576.0;
}

// Levels read by k_short2 / k_short_corr: every slice compact and coded,
// 1 to 8 slots per lane, and in the binary64 cycle at most 2^18 rows (the
// larger binary64 levels are bandwidth-bound and measured faster with
// k_sweep2, 160^3 solve 9.05 ms with this cap, 9.09 ms with 2^17 and 9.44 ms
// with none; the binary32 cycle is fastest with every level here, 7.27 ms
// against 7.44 ms with a 2^20 cap).
#ifndef AMG_SHORT_MAX_ROWS_F64
#define AMG_SHORT_MAX_ROWS_F64 262144
#endif
#ifndef AMG_SHORT_MAX_ROWS_F32
#define AMG_SHORT_MAX_ROWS_F32 0x7fffffff
#endif
template <class T>
bool short_coded(const Sell &S) {
  const int cap = sizeof(T) == 8 ? AMG_SHORT_MAX_ROWS_F64 : AMG_SHORT_MAX_ROWS_F32;
  return S.ndict > 0 && S.n <= cap && S.groups_compact * kSlice == S.nslots && S.wmin >= 1 && S.wmax <= 8;
}

// xw: store the new iterate widened to binary64 there instead of in xn.
template <class T>
void launch_sweep(const int *skip, const Level &L, const T *rhs, const T *x, T *xn, hipStream_t s,
                  double *xw = nullptr) {
  const int n = L.A.n;
  if (short_coded<T>(L.S)) {
    if (streamed<T>(L))
      hipLaunchKernelGGL((k_short2<T, true, false>), grid_for(n, 2 * kBlock), dim3(kBlock), 0, s, skip, n,
                         sell_ref(L.S), val_ref<T>(L.S), plain_pvals<T>(nullptr), rhs, x, xn, xw);
    else
      hipLaunchKernelGGL((k_short2<T, false, false>), grid_for(n, 2 * kBlock), dim3(kBlock), 0, s, skip, n,
                         sell_ref(L.S), val_ref<T>(L.S), plain_pvals<T>(nullptr), rhs, x, xn, xw);
    return;
  }
  if (L.S.ndict) {
    if (streamed<T>(L))
      hipLaunchKernelGGL((k_sweep2<T, true>), grid_for(n, 2 * kBlock), dim3(kBlock), 0, s, skip, n,
                         sell_ref(L.S), val_ref<T>(L.S), rhs, x, xn, xw);
    else
      hipLaunchKernelGGL((k_sweep2<T, false>), grid_for(n, 2 * kBlock), dim3(kBlock), 0, s, skip, n,
                         sell_ref(L.S), val_ref<T>(L.S), rhs, x, xn, xw);
    return;
  }
  if (streamed<T>(L))
    hipLaunchKernelGGL((k_sweep<T, true>), grid_for(n), dim3(kBlock), 0, s, skip, n, sell_ref(L.S),
                       val_ref<T>(L.S), rhs, x, xn, xw);
  else
    hipLaunchKernelGGL((k_sweep<T, false>), grid_for(n), dim3(kBlock), 0, s, skip, n, sell_ref(L.S),
                       val_ref<T>(L.S), rhs, x, xn, xw);
}

template <class T>
void launch_resid(const int *skip, const Level &L, const T *rhs, const T *x, T *t, hipStream_t s) {
  const int n = L.A.n;
  if (short_coded<T>(L.S)) {
    if (streamed<T>(L))
      hipLaunchKernelGGL((k_short2<T, true, true>), grid_for(n, 2 * kBlock), dim3(kBlock), 0, s, skip, n,
                         sell_ref(L.S), val_ref<T>(L.S), pvals_of<T>(L), rhs, x, t, nullptr);
    else
      hipLaunchKernelGGL((k_short2<T, false, true>), grid_for(n, 2 * kBlock), dim3(kBlock), 0, s, skip, n,
                         sell_ref(L.S), val_ref<T>(L.S), pvals_of<T>(L), rhs, x, t, nullptr);
    return;
  }
  if (L.S.ndict) {
    if (streamed<T>(L))
      hipLaunchKernelGGL((k_resid_scaled2<T, true>), grid_for(n, 2 * kBlock), dim3(kBlock), 0, s, skip,
                         n, sell_ref(L.S), val_ref<T>(L.S), pvals_of<T>(L), rhs, x, t);
    else
      hipLaunchKernelGGL((k_resid_scaled2<T, false>), grid_for(n, 2 * kBlock), dim3(kBlock), 0, s, skip,
                         n, sell_ref(L.S), val_ref<T>(L.S), pvals_of<T>(L), rhs, x, t);
    return;
  }
  if (streamed<T>(L))
    hipLaunchKernelGGL((k_resid_scaled<T, true>), grid_for(n), dim3(kBlock), 0, s, skip, n,
                       sell_ref(L.S), val_ref<T>(L.S), pval_of<T>(L), rhs, x, t);
  else
    hipLaunchKernelGGL((k_resid_scaled<T, false>), grid_for(n), dim3(kBlock), 0, s, skip, n,
                       sell_ref(L.S), val_ref<T>(L.S), pval_of<T>(L), rhs, x, t);
}

// Prolongation fused into the first post-sweep: 0 never, 1 on levels of at
// most kFuseMaxRows rows, whose kernels are launch- and latency-bound (on
// larger levels the four gathers per slot of the fused kernel cost more
// than the separate vector pass), 2 always.
#ifndef AMG_FUSE_PROLONG
#define AMG_FUSE_PROLONG 1
#endif
constexpr int kFuseMaxRows = 131072;
// x + P e followed by one sweep, xn the result (A: level k, e: level k+1 output).
template <class T>
void launch_corr_sweep(const int *skip, const Level &L, const T *rhs, const T *e, T *x, T *xn,
                       hipStream_t s) {
  const int n = L.A.n;
  if (AMG_FUSE_PROLONG == 0 || (AMG_FUSE_PROLONG == 1 && n > kFuseMaxRows)) {
    hipLaunchKernelGGL(k_prolong<T>, grid_for(n), dim3(kBlock), 0, s, skip, n, L.agg.p, pvals_of<T>(L),
                       e, x);
    launch_sweep<T>(skip, L, rhs, x, xn, s);
  } else if (short_coded<T>(L.S)) {
    hipLaunchKernelGGL(k_short_corr<T>, grid_for(n), dim3(kBlock), 0, s, skip, n, sell_ref(L.S),
                       val_ref<T>(L.S), rhs, x, L.agg.p, pval_of<T>(L), e, xn);
  } else if (streamed<T>(L)) {
    hipLaunchKernelGGL((k_sweep_corr<T, true>), grid_for(n), dim3(kBlock), 0, s, skip, n,
                       sell_ref(L.S), val_ref<T>(L.S), rhs, x, L.agg.p, pval_of<T>(L), e, xn);
  } else {
    hipLaunchKernelGGL((k_sweep_corr<T, false>), grid_for(n), dim3(kBlock), 0, s, skip, n,
                       sell_ref(L.S), val_ref<T>(L.S), rhs, x, L.agg.p, pval_of<T>(L), e, xn);
  }
}

#ifndef AMG_SHORT_RESTRICT
#define AMG_SHORT_RESTRICT 1
#endif
// One-pass restriction on levels of at most kFuseRestrictRows rows;
// returns false (nothing launched) on larger levels.
#ifndef AMG_FUSE_RESTRICT_ROWS
#define AMG_FUSE_RESTRICT_ROWS 131072
#endif
constexpr int kFuseRestrictRows = AMG_FUSE_RESTRICT_ROWS;
template <class T>
bool launch_resid_agg(const amg_hierarchy *h, const int *skip, const Level &L, const T *rhs, const T *x,
                      T *rc, const T *dinvc, T *xc) {
  if (L.A.n > kFuseRestrictRows) return false;
  const int steps = h->p.aggr_steps;   // aggregates of at most 2^steps members
  const int64_t nc = L.nc;
  hipStream_t s = h->stream;
  const bool shortr = AMG_SHORT_RESTRICT && L.S.wmax <= 8;   // every row at most 8 entries
#define AMG_RA(G, S)                                                                                      \
  hipLaunchKernelGGL((k_resid_agg<T, G, S>), grid_for(nc * G), dim3(kBlock), 0, s, skip, L.nc, L.mptr.p,   \
                     L.mem.p, L.A.rp.p, L.A.ci.p, L.A.v.p, pval_of<T>(L), rhs, x, rc, dinvc, xc)
#define AMG_RA2(G)        \
  if (shortr) AMG_RA(G, true); \
  else AMG_RA(G, false)
  if (steps <= 1) { AMG_RA2(2); }
  else if (steps == 2) { AMG_RA2(4); }
  else if (steps == 3) { AMG_RA2(8); }
  else { AMG_RA2(16); }
#undef AMG_RA2
#undef AMG_RA
  return true;
}

void launch_spmv(const Level &L, const double *x, double *y, hipStream_t s) {
  const int n = L.A.n;
  if (streamed<double>(L))
    hipLaunchKernelGGL((k_spmv<double, true>), grid_for(n), dim3(kBlock), 0, s, n, sell_ref(L.S),
                       val_ref<double>(L.S), x, y);
  else
    hipLaunchKernelGGL((k_spmv<double, false>), grid_for(n), dim3(kBlock), 0, s, n, sell_ref(L.S),
                       val_ref<double>(L.S), x, y);
}

// Where level k puts the first smoothing iterate so that, after all its
// ping-pong sweeps, the level's result lands in `out`.  nullptr when the
// level has no first sweep (direct coarsest solve, or no pre-smoothing) or
// runs in the coarse-tail kernel, which forms its own.
template <class T>
T *first_buffer(amg_hierarchy *h, int k, T *out) {
  Level &L = h->L[k];
  const amg_params &P = h->p;
  if (k >= h->tail_start) return nullptr;
  if (k == static_cast<int>(h->L.size()) - 1) {
    // the binary32 cycle's coarsest sweeps run in binary64 and form their own first iterate
    if (h->coarse_dense || std::is_same<T, float>::value) return nullptr;
    return ((P.coarse_sweeps - 1) % 2 == 0) ? out : tbuf<T>(L);
  }
  if (P.pre_sweeps == 0) return nullptr;
  const int swaps = (P.pre_sweeps - 1) + P.post_sweeps;
  return (swaps % 2 == 0) ? out : tbuf<T>(L);
}

// Level k of the V-cycle in precision T; the result lands in `out`.
// first_done: the first smoothing iterate is already in first_buffer(k).
// wide (binary32 fine level only): when the level ends with a plain sweep,
// that sweep stores the result widened to binary64 there instead of in out,
// and the call returns true.
template <class T>
bool vcycle_level(amg_hierarchy *h, const int *skip, int k, const T *rhs, T *out, bool first_done,
                  double *wide = nullptr) {
  hipStream_t s = h->stream;
  Level &L = h->L[k];
  const int n = L.A.n;
  const int nl = static_cast<int>(h->L.size());
  const amg_params &P = h->p;
  if (k >= h->tail_start) {
    auto kern = (h->tail_w <= 8) ? k_vcycle_tail<T, 8> : k_vcycle_tail<T, 16>;
    hipLaunchKernelGGL(kern, dim3(1), dim3(kTailThreads), 0, s, skip, nl - k,
                       tail_desc<T>(h) + (k - h->tail_start), h->Ainv.p, h->coarse_dense,
                       P.pre_sweeps, P.post_sweeps, P.coarse_sweeps, rhs, out);
    return false;
  }
  if (k == nl - 1 && std::is_same<T, float>::value) {
    // Mixed precision: the coarsest solve stays in binary64 (sweeps on the
    // binary64 matrix and l1 diagonal from the widened right-hand side; the
    // result is rounded back to binary32).
    double *A = L.x.p, *B = L.t.p;
    if ((P.coarse_sweeps - 1) % 2 != 0) std::swap(A, B);
    hipLaunchKernelGGL(k_f2d_first, grid_for(n), dim3(kBlock), 0, s, skip, n,
                       reinterpret_cast<const float *>(rhs), L.dinv.p, L.r.p, A);
    for (int q = 1; q < P.coarse_sweeps; ++q) { launch_sweep<double>(skip, L, L.r.p, A, B, s); std::swap(A, B); }
    hipLaunchKernelGGL(k_d2f, grid_for(n), dim3(kBlock), 0, s, skip, n, A, reinterpret_cast<float *>(out));
    return false;
  }
  if (k == nl - 1) {
    {
      T *A = first_buffer<T>(h, k, out);
      T *B = (A == out) ? tbuf<T>(L) : out;
      if (!first_done)
        hipLaunchKernelGGL(k_sweep_first<T>, grid_for(n), dim3(kBlock), 0, s, skip, n, dinv_of<T>(L),
                           rhs, A);
      for (int q = 1; q < P.coarse_sweeps; ++q) { launch_sweep<T>(skip, L, rhs, A, B, s); std::swap(A, B); }
    }
    return false;
  }
  const int swaps = (P.pre_sweeps > 0 ? P.pre_sweeps - 1 : 0) + P.post_sweeps;
  T *A = (swaps % 2 == 0) ? out : tbuf<T>(L);
  T *B = (A == out) ? tbuf<T>(L) : out;
  if (P.pre_sweeps == 0) {
    hipLaunchKernelGGL(k_zero<T>, grid_for(n), dim3(kBlock), 0, s, skip, n, A);
  } else {
    if (!first_done)
      hipLaunchKernelGGL(k_sweep_first<T>, grid_for(n), dim3(kBlock), 0, s, skip, n, dinv_of<T>(L),
                         rhs, A);
    for (int q = 1; q < P.pre_sweeps; ++q) { launch_sweep<T>(skip, L, rhs, A, B, s); std::swap(A, B); }
  }
  // restriction of the residual; B is free until the first post-sweep
  Level &C = h->L[k + 1];
  T *xc = first_buffer<T>(h, k + 1, xbuf<T>(C));
  if (!launch_resid_agg<T>(h, skip, L, rhs, A, rbuf<T>(C), dinv_of<T>(C), xc)) {
    launch_resid<T>(skip, L, rhs, A, B, s);
    hipLaunchKernelGGL(k_agg_sum<T>, grid_for(L.nc), dim3(kBlock), 0, s, skip, L.nc, L.mptr.p, L.mem.p,
                       B, rbuf<T>(C), dinv_of<T>(C), xc);
  }
  vcycle_level<T>(h, skip, k + 1, rbuf<T>(C), xbuf<T>(C), xc != nullptr);
  if (P.post_sweeps == 0) {
    hipLaunchKernelGGL(k_prolong<T>, grid_for(n), dim3(kBlock), 0, s, skip, n, L.agg.p, pvals_of<T>(L),
                       xbuf<T>(C), A);
    return false;
  }
  launch_corr_sweep<T>(skip, L, rhs, xbuf<T>(C), A, B, s);
  std::swap(A, B);
  for (int q = 1; q < P.post_sweeps; ++q) {
    launch_sweep<T>(skip, L, rhs, A, B, s, q + 1 == P.post_sweeps ? wide : nullptr);
    std::swap(A, B);
  }
  return wide != nullptr && P.post_sweeps >= 2;
}

// ---------------------------------- general cycle (Appendix A options)
// H- and W-cycles and the Jacobi / Gauss-Seidel smoothers, in binary64.
// Coarse-grid corrections per visit of level k: 1 (V), 2 (W), 2 on odd
// levels and 1 on even ones (H); with two, the coarse system is
// approximated by two cycles from zero: e = C(r_c), e += C(r_c - A_c e).
// Smoothers: l1-Jacobi and Jacobi sweep x <- x + dinv (r - A x) with dinv =
// 1 / sum_j |a_ij| or 1 / a_ii (from zero: x = dinv r, then nu - 1 sweeps);
// Gauss-Seidel passes update x_i <- x_i + (r_i - sum_j a_ij x_j) / a_ii in
// place, row by row (from zero: x = 0, then nu passes); FGS/BGS runs forward
// passes before the correction and backward ones after it (alternating,
// forward first, on the coarsest level); symmetrized GS a forward and a
// backward pass per sweep.  Rows are folded in CSR order.
//
// A Gauss-Seidel pass runs as a level schedule: level(i) = 1 + the largest
// level of a stored neighbour j < i (0 without one).  Rows of one level have
// no stored entry between them, so they update concurrently; a forward
// pass takes the levels in ascending order, a backward pass in descending
// order (a neighbour j > i of row i always has a higher level), which gives
// exactly the sequential pass.
__global__ void k_sub_from(const int *skip, int n, const double *__restrict__ r, double *__restrict__ t) {
  AMG_SKIP_IF_DONE();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = r[i] - t[i];
}

__global__ void k_add_to(const int *skip, int n, double *__restrict__ z, const double *__restrict__ e) {
  AMG_SKIP_IF_DONE();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = z[i] + e[i];
}

__global__ void k_div_by(const int *skip, int n, double *z, double m) {
  AMG_SKIP_IF_DONE();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = z[i] / m;
}

__global__ void k_copy(const int *skip, int n, const double *__restrict__ a, double *__restrict__ b) {
  AMG_SKIP_IF_DONE();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// xn = x + dinv (r - A x) over the canonical CSR rows.
__global__ void __launch_bounds__(kBlock) k_csr_sweep(const int *skip, int n, const int *__restrict__ rp,
                                                      const int *__restrict__ ci,
                                                      const double *__restrict__ v,
                                                      const double *__restrict__ dinv,
                                                      const double *__restrict__ r,
                                                      const double *__restrict__ x, double *__restrict__ xn) {
  AMG_SKIP_IF_DONE();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) acc = acc + v[k] * x[ci[k]];
  xn[i] = x[i] + dinv[i] * (r[i] - acc);
}

__device__ __forceinline__ void gs_row(int i, const int *__restrict__ rp, const int *__restrict__ ci,
                                       const double *__restrict__ v, const double *__restrict__ dj,
                                       const double *__restrict__ r, double *x) {
  double acc = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) acc = acc + v[k] * x[ci[k]];
  x[i] = x[i] + dj[i] * (r[i] - acc);
}

// One level of a Gauss-Seidel pass: rows[0 .. cnt) are independent.
__global__ void __launch_bounds__(kBlock) k_gs_level(const int *skip, int cnt, const int *__restrict__ rows,
                                                     const int *__restrict__ rp, const int *__restrict__ ci,
                                                     const double *__restrict__ v,
                                                     const double *__restrict__ dj,
                                                     const double *__restrict__ r, double *x) {
  AMG_SKIP_IF_DONE();
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < cnt) gs_row(rows[q], rp, ci, v, dj, r, x);
}

// A whole Gauss-Seidel pass in one workgroup (small levels): the levels in
// order with a workgroup barrier between them.
constexpr int kGsSmallRows = 65536;
constexpr int kGsThreads = 1024;
__global__ void __launch_bounds__(kGsThreads) k_gs_pass_small(const int *skip, int nlev,
                                                              const int *__restrict__ ptr,
                                                              const int *__restrict__ rows,
                                                              const int *__restrict__ rp,
                                                              const int *__restrict__ ci,
                                                              const double *__restrict__ v,
                                                              const double *__restrict__ dj,
                                                              const double *__restrict__ r, double *x,
                                                              int forward) {
  AMG_SKIP_IF_DONE();
  for (int l0 = 0; l0 < nlev; ++l0) {
    const int l = forward ? l0 : nlev - 1 - l0;
    for (int q = ptr[l] + static_cast<int>(threadIdx.x); q < ptr[l + 1]; q += kGsThreads)
      gs_row(rows[q], rp, ci, v, dj, r, x);
    __syncthreads();
  }
}

// Level schedule, fixed point of level(i) = max over stored j < i of
// level(j) + 1: updated in place (relaxed atomic accesses) until a pass
// changes nothing; the fixed point is unique whatever order rows are seen in.
__global__ void __launch_bounds__(kBlock) k_gs_levels(int n, const int *__restrict__ rp,
                                                      const int *__restrict__ ci, int *lev, int *changed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int m = 0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = ci[k];
    if (j < i) m = max(m, __hip_atomic_load(lev + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1);
  }
  if (m > __hip_atomic_load(lev + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    __hip_atomic_store(lev + i, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicOr(changed, 1);
  }
}

__global__ void k_gs_count(int n, const int *__restrict__ lev, int *cnt, int *maxlev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicAdd(cnt + lev[i], 1);
  atomicMax(maxlev, lev[i]);
}

// rows grouped by level (the order inside a level is free: its rows are independent)
__global__ void k_gs_place(int n, const int *__restrict__ lev, const int *__restrict__ ptr, int *fill,
                           int *rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int l = lev[i];
  rows[ptr[l] + atomicAdd(fill + l, 1)] = i;
}

__global__ void k_jacobi_diag(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                              const double *__restrict__ v, double *dj) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k)
    if (ci[k] == i) d = v[k];
  dj[i] = 1.0 / d;
}

bool general_cycle(const amg_hierarchy *h) {
  const amg_params &P = h->p;
  return P.precond && (P.cycle_type != AMG_CYCLE_V || P.relax_type != AMG_RELAX_L1_JACOBI ||
                       P.coarse_relax != AMG_RELAX_L1_JACOBI);
}

int corrections(const amg_hierarchy *h, int k) {
  if (h->p.cycle_type == AMG_CYCLE_W) return 2;
  if (h->p.cycle_type == AMG_CYCLE_H) return (k % 2 == 1) ? 2 : 1;
  return 1;
}

void gs_pass(amg_hierarchy *h, const int *skip, Level &L, const double *r, double *x, bool forward) {
  hipStream_t s = h->stream;
  const int n = L.A.n;
  const int nlev = static_cast<int>(L.gs_ptr.size()) - 1;
  if (n <= kGsSmallRows) {
    hipLaunchKernelGGL(k_gs_pass_small, dim3(1), dim3(kGsThreads), 0, s, skip, nlev, L.gs_ptr_d.p,
                       L.gs_rows.p, L.A.rp.p, L.A.ci.p, L.A.v.p, L.djac.p, r, x, forward ? 1 : 0);
    return;
  }
  for (int l0 = 0; l0 < nlev; ++l0) {
    const int l = forward ? l0 : nlev - 1 - l0;
    const int cnt = L.gs_ptr[l + 1] - L.gs_ptr[l];
    hipLaunchKernelGGL(k_gs_level, grid_for(cnt), dim3(kBlock), 0, s, skip, cnt,
                       L.gs_rows.p + L.gs_ptr[l], L.A.rp.p, L.A.ci.p, L.A.v.p, L.djac.p, r, x);
  }
}

// nsw further sweeps of smoother `type` on level k, in place on x; pass: +1
// pre-smoothing, -1 post-smoothing, 0 the coarsest level.
void smooth_more_g(amg_hierarchy *h, const int *skip, int k, int type, int pass, const double *r, int nsw,
                   double *x) {
  hipStream_t s = h->stream;
  Level &L = h->L[k];
  const int n = L.A.n;
  if (type == AMG_RELAX_L1_JACOBI || type == AMG_RELAX_JACOBI) {
    const double *d = (type == AMG_RELAX_L1_JACOBI) ? L.dinv.p : L.djac.p;
    double *a = x, *b = L.t.p;
    for (int q = 0; q < nsw; ++q) {
      if (type == AMG_RELAX_L1_JACOBI)   // the V-cycle's sweep kernels: the same fold and 1 / l1 bits
        launch_sweep<double>(skip, L, r, a, b, s);
      else
        hipLaunchKernelGGL(k_csr_sweep, grid_for(n), dim3(kBlock), 0, s, skip, n, L.A.rp.p, L.A.ci.p,
                           L.A.v.p, d, r, a, b);
      std::swap(a, b);
    }
    if (a != x) hipLaunchKernelGGL(k_copy, grid_for(n), dim3(kBlock), 0, s, skip, n, a, x);
    return;
  }
  for (int q = 0; q < nsw; ++q) {
    if (type == AMG_RELAX_GS) {
      gs_pass(h, skip, L, r, x, pass > 0 || (pass == 0 && q % 2 == 0));
    } else {
      gs_pass(h, skip, L, r, x, true);
      gs_pass(h, skip, L, r, x, false);
    }
  }
}

void smooth_zero_g(amg_hierarchy *h, const int *skip, int k, int type, int pass, const double *r, int nsw,
                   double *x) {
  hipStream_t s = h->stream;
  Level &L = h->L[k];
  const int n = L.A.n;
  if (nsw <= 0 || type == AMG_RELAX_GS || type == AMG_RELAX_SYM_GS) {
    hipLaunchKernelGGL(k_zero<double>, grid_for(n), dim3(kBlock), 0, s, skip, n, x);
    if (nsw > 0) smooth_more_g(h, skip, k, type, pass, r, nsw, x);
    return;
  }
  const double *d = (type == AMG_RELAX_L1_JACOBI) ? L.dinv.p : L.djac.p;
  hipLaunchKernelGGL(k_sweep_first<double>, grid_for(n), dim3(kBlock), 0, s, skip, n, d, r, x);
  smooth_more_g(h, skip, k, type, pass, r, nsw - 1, x);
}

void cycle_general(amg_hierarchy *h, const int *skip, int k, const double *rhs, double *out) {
  hipStream_t s = h->stream;
  Level &L = h->L[k];
  const int n = L.A.n;
  const int nl = static_cast<int>(h->L.size());
  const amg_params &P = h->p;
  if (h->tail_general && k >= h->tail_start) {   // this level and all below in one workgroup
    auto kern = (h->tail_w <= 8) ? k_cycle_tail_g<8> : k_cycle_tail_g<16>;
    hipLaunchKernelGGL(kern, dim3(1), dim3(kTailThreads), 0, s, skip, nl - k, k, P.cycle_type,
                       tail_desc<double>(h) + (k - h->tail_start), h->Ainv.p, h->coarse_dense,
                       P.pre_sweeps, P.post_sweeps, P.coarse_sweeps, rhs, out);
    AMG_LAUNCH_CHECK();
    return;
  }
  if (k == nl - 1) {
    if (h->coarse_dense) {   // the coarse-tail kernel holding only this level: z = A^-1 r
      auto kern = (h->tail_w <= 8) ? k_vcycle_tail<double, 8> : k_vcycle_tail<double, 16>;
      hipLaunchKernelGGL(kern, dim3(1), dim3(kTailThreads), 0, s, skip, 1, tail_desc<double>(h), h->Ainv.p,
                         h->coarse_dense, P.pre_sweeps, P.post_sweeps, P.coarse_sweeps, rhs, out);
    } else {
      smooth_zero_g(h, skip, k, P.coarse_relax, 0, rhs, P.coarse_sweeps, L.x.p);
      hipLaunchKernelGGL(k_copy, grid_for(n), dim3(kBlock), 0, s, skip, n, L.x.p, out);
    }
    return;
  }
  smooth_zero_g(h, skip, k, P.relax_type, 1, rhs, P.pre_sweeps, L.x.p);
  launch_resid<double>(skip, L, rhs, L.x.p, L.t.p, s);
  Level &C = h->L[k + 1];
  const int nc = L.nc;
  hipLaunchKernelGGL(k_agg_sum<double>, grid_for(nc), dim3(kBlock), 0, s, skip, nc, L.mptr.p, L.mem.p, L.t.p,
                     C.r.p, nullptr, nullptr);
  cycle_general(h, skip, k + 1, C.r.p, C.ge.p);
  for (int g = 1; g < corrections(h, k); ++g) {
    launch_spmv(C, C.ge.p, C.gw.p, s);
    hipLaunchKernelGGL(k_sub_from, grid_for(nc), dim3(kBlock), 0, s, skip, nc, C.r.p, C.gw.p);
    cycle_general(h, skip, k + 1, C.gw.p, C.gz.p);
    hipLaunchKernelGGL(k_add_to, grid_for(nc), dim3(kBlock), 0, s, skip, nc, C.ge.p, C.gz.p);
  }
  hipLaunchKernelGGL(k_prolong<double>, grid_for(n), dim3(kBlock), 0, s, skip, n, L.agg.p, pvals_of<double>(L), C.ge.p,
                     L.x.p);
  smooth_more_g(h, skip, k, P.relax_type, -1, rhs, P.post_sweeps, L.x.p);
  hipLaunchKernelGGL(k_copy, grid_for(n), dim3(kBlock), 0, s, skip, n, L.x.p, out);
  AMG_LAUNCH_CHECK();
}

// Setup of the general cycle's data: 1 / a_ii, Gauss-Seidel level schedules
// and the coarse-correction vectors.
void prepare_general(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  const amg_params &P = h->p;
  const int nl = static_cast<int>(h->L.size());
  const bool gs_smooth = P.relax_type == AMG_RELAX_GS || P.relax_type == AMG_RELAX_SYM_GS;
  const bool gs_coarse = !h->coarse_dense && (P.coarse_relax == AMG_RELAX_GS || P.coarse_relax == AMG_RELAX_SYM_GS);
  for (int k = 0; k < nl; ++k) {
    Level &L = h->L[k];
    const int n = L.A.n;
    L.djac.alloc(n);
    hipLaunchKernelGGL(k_jacobi_diag, grid_for(n), dim3(kBlock), 0, s, n, L.A.rp.p, L.A.ci.p, L.A.v.p, L.djac.p);
    AMG_LAUNCH_CHECK();
    if (k > 0) { L.ge.alloc(n); L.gw.alloc(n); L.gz.alloc(n); }
    const bool want_gs = (k < nl - 1) ? gs_smooth : gs_coarse;
    if (!want_gs) continue;
    dvec<int> lev(n), changed(1), cnt(n + 1), maxlev(1), fill(n + 1);
    hipLaunchKernelGGL(k_zero<int>, grid_for(n), dim3(kBlock), 0, s, nullptr, n, lev.p);
    for (int it = 0;; ++it) {
      if (it > n + 1) fail(AMG_ERR_DEVICE, "Gauss-Seidel level schedule did not settle");
      hipLaunchKernelGGL(k_zero<int>, dim3(1), dim3(kBlock), 0, s, nullptr, 1, changed.p);
      hipLaunchKernelGGL(k_gs_levels, grid_for(n), dim3(kBlock), 0, s, n, L.A.rp.p, L.A.ci.p, lev.p, changed.p);
      AMG_LAUNCH_CHECK();
      int c = 0;
      AMG_HIP(hipMemcpyAsync(&c, changed.p, sizeof(int), hipMemcpyDeviceToHost, s));
      AMG_HIP(hipStreamSynchronize(s));
      if (!c) break;
    }
    hipLaunchKernelGGL(k_zero<int>, grid_for(n + 1), dim3(kBlock), 0, s, nullptr, n + 1, cnt.p);
    hipLaunchKernelGGL(k_zero<int>, grid_for(n + 1), dim3(kBlock), 0, s, nullptr, n + 1, fill.p);
    hipLaunchKernelGGL(k_zero<int>, dim3(1), dim3(kBlock), 0, s, nullptr, 1, maxlev.p);
    hipLaunchKernelGGL(k_gs_count, grid_for(n), dim3(kBlock), 0, s, n, lev.p, cnt.p, maxlev.p);
    AMG_LAUNCH_CHECK();
    int ml = 0;
    AMG_HIP(hipMemcpyAsync(&ml, maxlev.p, sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    const int nlev = ml + 1;
    L.gs_ptr_d.alloc(nlev + 1);
    device_exclusive_scan(cnt.p, L.gs_ptr_d.p, nlev, s);
    L.gs_rows.alloc(n);
    hipLaunchKernelGGL(k_gs_place, grid_for(n), dim3(kBlock), 0, s, n, lev.p, L.gs_ptr_d.p, fill.p, L.gs_rows.p);
    AMG_LAUNCH_CHECK();
    L.gs_ptr.resize(nlev + 1);
    AMG_HIP(hipMemcpyAsync(L.gs_ptr.data(), L.gs_ptr_d.p, sizeof(int) * (nlev + 1), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
  }
}

// Mixed precision: the residual is rounded to binary32 on entry (fused with
// the first sweep), the cycle runs in binary32 except for the coarsest solve
// (binary64 inside its kernel), and the result is widened to binary64.
void vcycle_mixed(amg_hierarchy *h, const int *skip, const double *r, double *z, bool first_done) {
  hipStream_t s = h->stream;
  Level &L = h->L[0];
  const int n = L.A.n;
  if (h->L.size() == 1) {   // single level: the direct solve in binary64
    vcycle_level<double>(h, skip, 0, r, z, false);
    return;
  }
  float *x1 = first_buffer<float>(h, 0, L.xf.p);
  if (!first_done)
    hipLaunchKernelGGL(k_d2f_first, grid_for(n), dim3(kBlock), 0, s, skip, n, r, L.dinvf.p, L.rf.p, x1);
  if (!vcycle_level<float>(h, skip, 0, L.rf.p, L.xf.p, x1 != nullptr, z))
    hipLaunchKernelGGL(k_f2d, grid_for(n), dim3(kBlock), 0, s, skip, n, L.xf.p, z);
}

// first_done: the residual kernel already wrote the first smoothing iterate
// (the outputs described by first_out_for).
// binary64: the binary64 cycle also in a mixed-precision hierarchy (the
// bootstrap's rate estimates belong to the setup, which is binary64).
void vcycle_any(amg_hierarchy *h, const int *skip, const double *r, double *z,
                bool first_done = false, bool binary64 = false) {
  const int n = h->L[0].A.n;
  if (!h->p.precond) {
    AMG_HIP(hipMemcpyAsync(z, r, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    return;
  }
  if (general_cycle(h)) cycle_general(h, skip, 0, r, z);
  else if (h->p.precision == AMG_PREC_MIXED && !binary64) vcycle_mixed(h, skip, r, z, first_done);
  else vcycle_level<double>(h, skip, 0, r, z, first_done);
  AMG_LAUNCH_CHECK();
}

// ------------------------------------------------- bootstrap composite
// Appendix A's bootstrap composite of hierarchies h (the first) and
// h->comp[0..]: multiplicative z = B_1 r, z += B_j (r - A z) for j = 2..m;
// symmetrized the same for j = 1..m and then j = m-1..1; additive
// z = (B_1 r + ... + B_m r) / m.  Residuals, sums and the division are
// binary64 in both precisions.
// z = B r for the composite of the first m hierarchies (m < 0: all of them);
// first_done as for vcycle_any (first hierarchy only).
void precond_apply(amg_hierarchy *h, const int *skip, const double *r, double *z, bool first_done,
                   int m = -1, bool binary64 = false) {
  const int total = 1 + static_cast<int>(h->comp.size());
  if (m < 0 || m > total) m = total;
  vcycle_any(h, skip, r, z, first_done, binary64);
  if (m <= 1 || !h->p.precond) return;
  hipStream_t s = h->stream;
  const int n = h->L[0].A.n;
  const int type = h->p.bootstrap_type;
  const int steps = (type == AMG_BOOTSTRAP_SYMMULT) ? 2 * m - 1 : m;
  for (int q = 1; q < steps; ++q) {
    const int j = (q < m) ? q : 2 * m - 2 - q;
    amg_hierarchy *c = (j == 0) ? h : h->comp[j - 1];
    // run on the head's stream (a capture stream while the head captures)
    const hipStream_t own = c->stream;
    c->stream = s;
    if (type == AMG_BOOTSTRAP_ADD) {
      vcycle_any(c, skip, r, h->ce.p, false, binary64);
    } else {
      launch_spmv(h->L[0], z, h->ct.p, s);
      hipLaunchKernelGGL(k_sub_from, grid_for(n), dim3(kBlock), 0, s, skip, n, r, h->ct.p);
      vcycle_any(c, skip, h->ct.p, h->ce.p, false, binary64);
    }
    c->stream = own;
    hipLaunchKernelGGL(k_add_to, grid_for(n), dim3(kBlock), 0, s, skip, n, z, h->ce.p);
  }
  if (type == AMG_BOOTSTRAP_ADD)
    hipLaunchKernelGGL(k_div_by, grid_for(n), dim3(kBlock), 0, s, skip, n, z, static_cast<double>(m));
  AMG_LAUNCH_CHECK();
}

// What the PCG residual kernels write for the next V-cycle whose output is z.
FirstOut first_out_for(amg_hierarchy *h, double *z) {
  FirstOut fo{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (!h->p.precond || general_cycle(h)) return fo;
  Level &L = h->L[0];
  if (h->p.precision == AMG_PREC_MIXED && h->L.size() > 1) {
    fo.rf = L.rf.p;
    fo.dinvf = L.dinvf.p;
    fo.xf = first_buffer<float>(h, 0, L.xf.p);
  } else {
    fo.dinv = L.dinv.p;
    fo.x = first_buffer<double>(h, 0, z);
  }
  return fo;
}

int nb_dot(int n) { return std::max(1, ceil_div(n, kBlock * kRowsDot)); }
int nb_upd(int n) { return std::max(1, ceil_div(n, kBlock * kRowsUpd)); }

// Device state of one PCG solve: the scalar block (with the `done` flag the
// iteration's kernels test) and 3 nb_dot(n) partial sums of the fine-level
// reductions.  The hierarchy's own buffers, or the allocation-free solve's
// static scratch.
struct PcgState {
  Scalars *sc;
  double *part;
};

PcgState own_state(amg_hierarchy *h) { return PcgState{h->sc.p, h->partials.p}; }

void launch_spmv_dots(amg_hierarchy *h, const int *skip, double *part) {
  const Level &L0 = h->L[0];
  const int n = L0.A.n, nbd = nb_dot(n);
  if (streamed<double>(L0))
    hipLaunchKernelGGL(k_pcg_spmv_dots<true>, dim3(nbd), dim3(kBlock), 0, h->stream, skip, n,
                       sell_ref(L0.S), val_ref<double>(L0.S), h->w.p, h->r.p, h->q.p, h->v.p, part);
  else
    hipLaunchKernelGGL(k_pcg_spmv_dots<false>, dim3(nbd), dim3(kBlock), 0, h->stream, skip, n,
                       sell_ref(L0.S), val_ref<double>(L0.S), h->w.p, h->r.p, h->q.p, h->v.p, part);
}

void enqueue_iteration(amg_hierarchy *h, PcgState ps) {
  hipStream_t s = h->stream;
  const Level &L0 = h->L[0];
  const int n = L0.A.n, nbd = nb_dot(n), nbu = nb_upd(n);
  const int *skip = &ps.sc->done;
  const FirstOut fo = first_out_for(h, h->w.p);
  precond_apply(h, skip, h->r.p, h->w.p, /*first_done=*/true);
  launch_spmv_dots(h, skip, ps.part);
  hipLaunchKernelGGL(k_pcg_dots_finish, dim3(1), dim3(kFinish), 0, s, skip, nbd, ps.part, ps.sc);
  hipLaunchKernelGGL(k_pcg_update, dim3(nbu), dim3(kBlock), 0, s, skip, n, h->w.p, h->v.p, h->d.p,
                     h->u.p, h->q.p, h->r.p, ps.sc, ps.part, fo);
  hipLaunchKernelGGL(k_pcg_norm_finish, dim3(1), dim3(kFinish), 0, s, skip, nbu, ps.part, ps.sc,
                     h->sc_host_dev);
  AMG_LAUNCH_CHECK();
}

// vectors: LDS vectors per row and level (4 for the V-cycle tail, 5 for the
// general cycle's)
template <class T>
void upload_tail(amg_hierarchy *h, dvec<unsigned char> &dst, bool fp32, int vectors) {
  std::vector<TailDesc<T>> D;
  int lds = 0;
  for (size_t k = h->tail_start; k < h->L.size(); ++k) {
    Level &L = h->L[k];
    TailDesc<T> t{};
    t.n = L.A.n;
    t.nc = L.nc;
    t.lds = lds;
    lds += vectors * L.A.n;
    t.sptr = L.S.sptr.p;
    t.col = L.S.col.p;
    t.val = val_ref<T>(L.S).val;   // the tail reads plain values
    t.pval = pval_of<T>(L);
    t.agg = L.agg.p;
    t.mptr = L.mptr.p;
    t.mem = L.mem.p;
    D.push_back(t);
  }
  if (lds > kTailLds) fail(AMG_ERR_DEVICE, "coarse tail exceeds its LDS budget");
  (void)fp32;
  dst.alloc(sizeof(TailDesc<T>) * std::max<size_t>(1, D.size()));
  if (!D.empty())
    AMG_HIP(hipMemcpyAsync(dst.p, D.data(), sizeof(TailDesc<T>) * D.size(), hipMemcpyHostToDevice,
                           h->stream));
  AMG_HIP(hipStreamSynchronize(h->stream));
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
  h->partials.alloc(static_cast<size_t>(nb_dot(n)) * 3);
  // The single-workgroup coarse tail: the longest suffix of levels with at
  // most kTailRows rows each whose vectors (4 per row) fit its LDS array.
  const int nl = static_cast<int>(h->L.size());
  h->tail_start = nl;
  int used = 0;
  // (the binary32 cycle solves a coarsest level without a direct solve by
  // binary64 sweeps, which the tail kernel does not provide; the general
  // cycle uses it for the direct coarsest solve only)
  const bool general = general_cycle(h);
  // the general cycle's own tail: l1-Jacobi smoothing everywhere, a direct
  // or l1-Jacobi coarsest solve (V/H/W); other smoothers run level by level
  h->tail_general = general && h->p.relax_type == AMG_RELAX_L1_JACOBI &&
                    (h->coarse_dense || h->p.coarse_relax == AMG_RELAX_L1_JACOBI);
  const int vectors = h->tail_general ? 5 : 4;
  const bool tail_ok = !(mixed && h->p.precond && !h->coarse_dense && nl > 1) && (!general || h->tail_general);
  // (a W-cycle visits the j-th tail level 2^j times: at most 12 levels, so
  // that one tail launch stays short whatever the hierarchy's depth)
  constexpr int kTailGeneralLevels = 12;
  for (int k = nl - 1; tail_ok && k >= 0; --k) {
    const int nk = h->L[k].A.n;
    if (nk > kTailRows || used + vectors * nk > kTailLds) break;
    if (h->tail_general && nl - k > kTailGeneralLevels) break;
    used += vectors * nk;
    h->tail_start = k;
  }
  if (general && !h->tail_general && h->coarse_dense) {
    h->tail_start = nl - 1;
    used = 4 * h->L[nl - 1].A.n;
  }
  if (h->coarse_dense && h->tail_start > nl - 1) fail(AMG_ERR_DEVICE, "dense coarsest level outside the tail");
  // widest slice of the tail levels: rows up to 8 slots stay in registers
  // whole, wider ones keep 16 there
  h->tail_w = 0;
  for (int k = h->tail_start; k < nl; ++k) {
    const Sell &S = h->L[k].S;
    std::vector<int> sp(S.nslices + 1);
    AMG_HIP(hipMemcpyAsync(sp.data(), S.sptr.p, sizeof(int) * sp.size(), hipMemcpyDeviceToHost, h->stream));
    AMG_HIP(hipStreamSynchronize(h->stream));
    for (int q = 0; q < S.nslices; ++q) h->tail_w = std::max(h->tail_w, (sp[q + 1] - sp[q]) / kSlice);
  }
  upload_tail<double>(h, h->tail_desc_d, false, vectors);
  if (mixed) upload_tail<float>(h, h->tail_desc_f, true, vectors);
  if (general) prepare_general(h);
  h->sc.alloc(1);
  AMG_HIP(hipMemsetAsync(h->sc.p, 0, sizeof(Scalars), h->stream));
  if (!h->sc_host) {
    AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->sc_host), sizeof(Scalars),
                          hipHostMallocMapped | hipHostMallocCoherent));
    AMG_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&h->sc_host_dev), h->sc_host, 0));
  }
}

void enqueue_vcycle(amg_hierarchy *h, const double *r, double *z) { precond_apply(h, nullptr, r, z, false); }

void enqueue_vcycle_single(amg_hierarchy *h, const double *r, double *z) { vcycle_any(h, nullptr, r, z); }

void enqueue_composite(amg_hierarchy *h, int m, const double *r, double *z) {
  precond_apply(h, nullptr, r, z, false, m, /*binary64=*/true);
}

void enqueue_spmv(amg_hierarchy *h, int k, const double *x, double *y) {
  launch_spmv(h->L[k], x, y, h->stream);
  AMG_LAUNCH_CHECK();
}

void enqueue_sweep(amg_hierarchy *h, int k, const double *r, const double *x, double *xn) {
  launch_sweep<double>(nullptr, h->L[k], r, x, xn, h->stream);
  AMG_LAUNCH_CHECK();
}

void destroy_graph(amg_hierarchy *h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
}

// Iterations the host keeps queued beyond the one it waits for.
#ifndef AMG_QUEUE_AHEAD
#define AMG_QUEUE_AHEAD 1
#endif
constexpr int kAhead = AMG_QUEUE_AHEAD;

// Alg. 1.  One iteration = one graph launch [V-cycle, v = A w + dots,
// scalars, vector updates + ||r||^2, convergence test, copy of the scalars
// to pinned host memory].  The host keeps one further iteration queued and
// waits on the older one; a queued iteration after convergence does nothing
// (and is not queued when the residual trend says the older one ends it).
//
// alloc_free: the iteration's kernels are launched one by one (no graph is
// instantiated) and the host waits by polling the scalars the last kernel of
// each iteration writes to pinned host memory (no events are created); the
// stream draining ends every wait, so it cannot outlast the queued work.
int pcg_run(amg_hierarchy *h, PcgState ps, bool alloc_free, const double *b, double *x, double rtol,
            int maxit, int *iters, double *relres) {
  hipStream_t s = h->stream;
  const Level &L0 = h->L[0];
  const int n = L0.A.n, nb = nb_dot(n);
  if (streamed<double>(L0))
    hipLaunchKernelGGL(k_pcg_init<true>, dim3(nb), dim3(kBlock), 0, s, n, sell_ref(L0.S), val_ref<double>(L0.S),
                       b, x, h->u.p, h->d.p, h->q.p, h->r.p, ps.part, first_out_for(h, h->w.p));
  else
    hipLaunchKernelGGL(k_pcg_init<false>, dim3(nb), dim3(kBlock), 0, s, n, sell_ref(L0.S), val_ref<double>(L0.S),
                       b, x, h->u.p, h->d.p, h->q.p, h->r.p, ps.part, first_out_for(h, h->w.p));
  hipLaunchKernelGGL(k_pcg_init_finish, dim3(1), dim3(kFinish), 0, s, nb, ps.part, ps.sc, rtol, maxit);
  AMG_LAUNCH_CHECK();
  Scalars st{};
  if (alloc_free) {   // the mirror starts from the initial state (polled below)
    AMG_HIP(hipMemcpyAsync(h->sc_host, ps.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    st = *h->sc_host;
  }
  if (alloc_free && !st.done) {
    const volatile Scalars *mirror = h->sc_host;
    // true once iteration j has ended (or the solve has), read from the mirror
    auto ended = [&](int j) { return mirror->done != 0 || mirror->it >= j; };
    int launched = 0;
    for (int k = 0; k <= kAhead && launched < maxit; ++k) {
      enqueue_iteration(h, ps);
      ++launched;
    }
    // as below for the graph path: no iteration queued behind one that the
    // residual trend says ends the solve (||r||^2 of the last two: rr_old,
    // rr_new)
    double rr_old = -1.0, rr_new = mirror->rr;
    const double thr2 = mirror->thr * mirror->thr;
    for (int j = 1;; ++j) {
      while (!ended(j)) {
        const hipError_t q = hipStreamQuery(s);
        if (q == hipSuccess) break;            // drained: the mirror holds the final state
        if (q != hipErrorNotReady) AMG_HIP(q);
      }
      if (mirror->done || j >= maxit) break;
      rr_old = rr_new;
      rr_new = mirror->rr;
      // iteration j + 1 must be queued; the one after it only if j + 1 is
      // not expected to end the solve
      const bool last = rr_old > 0.0 && rr_new * (rr_new / rr_old) <= 9.0 * thr2;
      if (launched < maxit && (launched <= j || !last)) {
        enqueue_iteration(h, ps);
        ++launched;
      }
    }
  } else if (!alloc_free) {
    // the first iterations are queued right behind the initial residual,
    // with no host round trip in between (they do nothing if it already
    // ended the solve: zero or non-finite right-hand side)
    if (h->use_graph && !h->graph_exec) {
      capture_graph(h->stream, &h->graph, [&] { enqueue_iteration(h, ps); });
      AMG_HIP(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
    }
    auto launch = [&]() {
      if (h->graph_exec) AMG_HIP(hipGraphLaunch(h->graph_exec, s));
      else enqueue_iteration(h, ps);
    };
    // iteration k (from 1) records ev[k % (kAhead + 1)]; before waiting on
    // iteration j at most j + kAhead have been launched, so its event is intact
    hipEvent_t ev[kAhead + 1];
    for (hipEvent_t &e : ev) AMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    int launched = 0;
    auto push = [&]() {
      launch();
      ++launched;
      AMG_HIP(hipEventRecord(ev[launched % (kAhead + 1)], s));
    };
    for (int k = 0; k < kAhead && launched < maxit; ++k) push();
    // ||r||^2 after the last two finished iterations (-1 while unknown)
    double rr_new = -1.0, rr_old = -1.0, thr2 = 0.0;
    for (int j = 1;; ++j) {
      // iteration j is queued; the next one is queued behind it unless j is
      // expected to end the solve (the residual norm extrapolated from the
      // last two within 3 rtol ||r_0||): an iteration queued after
      // convergence still dispatches every kernel of the graph
      const bool last = rr_old > 0.0 && rr_new * (rr_new / rr_old) <= 9.0 * thr2;
      if (launched < maxit && launched < j + kAhead && !last) push();
      AMG_HIP(hipEventSynchronize(ev[j % (kAhead + 1)]));
      const volatile Scalars *m = h->sc_host;
      if (m->done || j >= maxit) break;
      if (j == 1) {
        rr_new = m->nr0 * m->nr0;
        thr2 = m->thr * m->thr;
      }
      rr_old = rr_new;
      rr_new = m->rr;
      if (launched == j && launched < maxit) push();   // the one held back
    }
    // the solution copy goes behind whatever is still queued; the events
    // are destroyed once the stream has drained
    AMG_HIP(hipMemcpyAsync(x, h->u.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipStreamSynchronize(s));
    for (hipEvent_t &e : ev) (void)hipEventDestroy(e);
  }
  if (alloc_free) {
    AMG_HIP(hipMemcpyAsync(x, h->u.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipStreamSynchronize(s));
  }
  st = *h->sc_host;   // the scalars after the last iteration that ran
  *iters = st.it;
  *relres = (st.nr0 == 0.0) ? 0.0 : sqrt(st.rr) / st.nr0;
  if (st.status != 0) return st.status;
  if (st.nr0 == 0.0) return AMG_OK;
  return st.conv ? AMG_OK : AMG_NOT_CONVERGED;
}

int pcg_solve(amg_hierarchy *h, const double *b, double *x, double rtol, int maxit, int *iters,
              double *relres) {
  return pcg_run(h, own_state(h), false, b, x, rtol, maxit, iters, relres);
}

// ------------------------------------------------ allocation-free solve
// The PCG state of amg_pcg_solve_noalloc lives in this file-scope array, one
// copy per device, held until the process ends: the scalar block in the
// first 256 bytes, then the partial sums.  Host code never passes the
// array's name to a kernel; it uses the device address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
constexpr size_t kNoAllocBytes = size_t(4) << 20;
constexpr size_t kNoAllocHead = 256;
static_assert(sizeof(Scalars) <= kNoAllocHead, "scalar block exceeds its slot");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void *noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(AMG_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    AMG_HIP(hipGetDevice(&cur));
    if (cur != dev) AMG_HIP(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) AMG_HIP(hipSetDevice(cur));
    AMG_HIP(e);
    if (!p) fail(AMG_ERR_DEVICE, "no device address for the solve scratch");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

int64_t noalloc_max_rows() {
  const int64_t parts = static_cast<int64_t>((kNoAllocBytes - kNoAllocHead) / (3 * sizeof(double)));
  return parts * kBlock * kRowsDot;
}

int pcg_solve_noalloc(amg_hierarchy *h, const double *b, double *x, double rtol, int maxit,
                      int *iters, double *relres) {
  const int n = h->L[0].A.n;
  if (static_cast<int64_t>(n) > noalloc_max_rows())
    fail(AMG_ERR_INVALID, "amg_pcg_solve_noalloc: n = " + std::to_string(n) + " exceeds its scratch (" +
                              std::to_string(noalloc_max_rows()) + " rows)");
  unsigned char *base = static_cast<unsigned char *>(noalloc_scratch(h->dev));
  PcgState ps{reinterpret_cast<Scalars *>(base), reinterpret_cast<double *>(base + kNoAllocHead)};
  // the scalar block starts from zero (k_pcg_init_finish then sets every
  // field it reads); the partial sums are written before they are read
  hipLaunchKernelGGL(k_zero<double>, dim3(1), dim3(kBlock), 0, h->stream, nullptr,
                     static_cast<int>(kNoAllocHead / sizeof(double)), reinterpret_cast<double *>(base));
  AMG_LAUNCH_CHECK();
  return pcg_run(h, ps, true, b, x, rtol, maxit, iters, relres);
}

// ------------------------------------------------------- kernel timing
void time_kernel(amg_hierarchy *h, int kernel, int k, int reps, double *avg_ms, double *bytes) {
  hipStream_t s = h->stream;
  if (k < 0 || k >= static_cast<int>(h->L.size())) fail(AMG_ERR_INVALID, "level out of range");
  Level &L = h->L[k];
  const int n = L.A.n;
  const double nnz = static_cast<double>(L.A.nnz);
  const int nbu = nb_upd(n);
  const bool has_coarse = k + 1 < static_cast<int>(h->L.size());
  if ((kernel == 2 || kernel == 3 || kernel == 5) && !has_coarse) fail(AMG_ERR_INVALID, "no coarser level");
  if (kernel == 4 && k != 0) fail(AMG_ERR_INVALID, "the PCG update exists on level 0 only");
  if (kernel < 0 || kernel > 5) fail(AMG_ERR_INVALID, "unknown kernel id");
  auto launch = [&]() {
    switch (kernel) {
      case 0:
        if (k == 0) launch_spmv_dots(h, nullptr, h->partials.p);
        else launch_spmv(L, L.x.p, L.t.p, s);
        break;
      case 1:
        launch_sweep<double>(nullptr, L, L.r.p, L.x.p, L.t.p, s);
        break;
      case 2:
        launch_resid<double>(nullptr, L, L.r.p, L.x.p, L.t.p, s);
        hipLaunchKernelGGL(k_agg_sum<double>, grid_for(L.nc), dim3(kBlock), 0, s, nullptr, L.nc,
                           L.mptr.p, L.mem.p, L.t.p, h->L[k + 1].r.p, h->L[k + 1].dinv.p,
                           h->L[k + 1].x.p);
        break;
      case 3:
        hipLaunchKernelGGL(k_prolong<double>, grid_for(n), dim3(kBlock), 0, s, nullptr, n, L.agg.p,
                           pvals_of<double>(L), h->L[k + 1].x.p, L.t.p);
        break;
      case 5:
        launch_corr_sweep<double>(nullptr, L, L.r.p, h->L[k + 1].x.p, L.x.p, L.t.p, s);
        break;
      default:
        hipLaunchKernelGGL(k_pcg_update, dim3(nbu), dim3(kBlock), 0, s, nullptr, n, h->w.p, h->v.p,
                           h->d.p, h->u.p, h->q.p, h->r.p, h->sc.p, h->partials.p,
                           first_out_for(h, h->w.p));
        break;
    }
    AMG_LAUNCH_CHECK();
  };
  // defined, finite inputs for the timed launches (the PCG scalars are left
  // as the last solve set them, or zero)
  for (double *p : {L.x.p, L.r.p, L.t.p})
    hipLaunchKernelGGL(k_zero<double>, grid_for(n), dim3(kBlock), 0, s, nullptr, n, p);
  if (k == 0)
    for (double *p : {h->w.p, h->r.p, h->q.p, h->v.p, h->d.p, h->u.p})
      hipLaunchKernelGGL(k_zero<double>, grid_for(n), dim3(kBlock), 0, s, nullptr, n, p);
  if (has_coarse)
    hipLaunchKernelGGL(k_zero<double>, grid_for(L.nc), dim3(kBlock), 0, s, nullptr, L.nc,
                       h->L[k + 1].x.p);
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
  // algorithmic bytes: the matrix once in the form the kernel reads (values
  // or value codes and their table, column offsets or columns, group bases,
  // slice pointers), vectors once
  const double bv = 8.0, nd = static_cast<double>(n), ncd = static_cast<double>(L.nc);
  const Sell &S = L.S;
  const double idx = S.cdel.p ? 2.0 * S.nnz_compact + 4.0 * (nnz - S.nnz_compact) + 4.0 * S.groups_compact
                              : 4.0 * nnz;
  const double vbytes = S.ndict ? 1.0 * nnz + bv * S.ndict : bv * nnz;
  const double mat = vbytes + idx + 4.0 * (S.nslices + 1);
  const double pv = L.npdict ? 1.0 * nd + bv * L.npdict : bv * nd;   // P values, coded or not
  switch (kernel) {
    case 0: *bytes = mat + 2 * bv * nd + (k == 0 ? 2 * bv * nd : 0.0); break;
    case 1: *bytes = mat + 3 * bv * nd; break;
    case 2: *bytes = mat + 4 * bv * nd + pv + 4 * nd + 4 * (ncd + 1) + 3 * bv * ncd; break;
    case 3: *bytes = 2 * bv * nd + pv + 4 * nd + bv * ncd; break;
    case 5: *bytes = mat + 4 * bv * nd + 4 * nd + bv * ncd; break;
    case 4: {
      const FirstOut fo = first_out_for(h, h->w.p);
      *bytes = 10 * bv * nd + (fo.x ? 16 * nd : 0.0) + (fo.rf ? 4 * nd : 0.0) + (fo.xf ? 8 * nd : 0.0);
      break;
    }
  }
}

}  // namespace amg
