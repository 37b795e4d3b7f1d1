// Hierarchy construction on the GPU (Alg. 3 with the s-step composition of
// Sec. 3.1; matching of Sec. 4.1).  Every kernel is deterministic: results do
// not depend on workgroup scheduling, so aggregate maps, coarse patterns and
// coarse values are reproducible bit for bit.  Floating-point contraction is
// disabled for this library (-ffp-contract=off): each multiply and add rounds
// on its own, in the orders stated at each kernel.
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>
#include <type_traits>
#include <utility>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "amg_internal.hpp"

namespace amg {

namespace {

constexpr int kFree = -2;    // matching state: not yet decided
constexpr int kSingle = -1;  // no partner (also the exported value)

inline dim3 grid_for(int64_t n, int block = kBlock) {
  return dim3(static_cast<unsigned>(std::max<int64_t>(1, (n + block - 1) / block)));
}

// ------------------------------------------------------------------- scan
// Exclusive prefix sum of int32 counts; out has n+1 entries, out[n] = total.
__global__ void k_scan_tiles(const int *in, int *out, int *tile_sum, int n) {
  constexpr int kItems = 4, kTile = kBlock * kItems;
  __shared__ int wsum[kBlock / kWave];
  const int base = blockIdx.x * kTile + threadIdx.x * kItems;
  int v[kItems], local = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    local += v[j];
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int incl = local;
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  int woff = 0;
  for (int q = 0; q < wid; ++q) woff += wsum[q];
  int run = woff + incl - local;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == kBlock - 1) tile_sum[blockIdx.x] = woff + incl;
}

__global__ void k_scan_add(int *out, const int *tile_off, int n) {
  constexpr int kTile = kBlock * 4;
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] += tile_off[i / kTile];
}

__global__ void k_set_total(int *out, int n, const int *tile_off, const int *tile_sum, int ntiles) {
  out[n] = tile_off[ntiles - 1] + tile_sum[ntiles - 1];
}

__global__ void k_fill_int(int n, int *a, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

constexpr int kScanTile = kBlock * 4;

// Scan of n ints with tile sums and offsets carved from `scratch` (each
// recursion level takes 2 ntiles + 1 ints, then passes the rest on).
void scan_impl(const int *in, int *out, int n, hipStream_t s, int *scratch) {
  const int ntiles = std::max(1, ceil_div(n, kScanTile));
  int *tsum = scratch, *toff = scratch + ntiles;
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kBlock), 0, s, in, out, tsum, n);
  AMG_LAUNCH_CHECK();
  if (ntiles > 1) {
    scan_impl(tsum, toff, ntiles, s, toff + ntiles + 1);
    hipLaunchKernelGGL(k_scan_add, grid_for(n), dim3(kBlock), 0, s, out, toff, n);
    AMG_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, 1, toff, 0);
  }
  hipLaunchKernelGGL(k_set_total, dim3(1), dim3(1), 0, s, out, n, toff, tsum, ntiles);
  AMG_LAUNCH_CHECK();
}

// Scratch ints a scan of n entries needs over all recursion levels.
size_t scan_scratch_ints(int n) {
  size_t total = 0;
  for (int m = n;;) {
    const int nt = std::max(1, ceil_div(m, kScanTile));
    total += 2 * static_cast<size_t>(nt) + 1;
    if (nt == 1) break;
    m = nt;
  }
  return total;
}

// Per-thread, per-device grow-only scan scratch (scans of one thread are
// ordered on its streams; the buffer lives until the thread ends).
int *scan_scratch(int n) {
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  thread_local std::vector<dvec<int>> bufs;
  if (static_cast<int>(bufs.size()) <= dev) bufs.resize(dev + 1);
  const size_t need = scan_scratch_ints(n);
  if (bufs[dev].n < need) {
    NoPool plain;   // the cache outlives any one setup and its stream
    bufs[dev].alloc(std::max<size_t>(need, 1 << 16));
  }
  return bufs[dev].p;
}

void exclusive_scan(const int *in, int *out, int n, hipStream_t s) {
  scan_impl(in, out, n, s, scan_scratch(n));
}

// Small device-to-host reads go through a per-thread pinned buffer (a copy
// into pageable memory is staged by the runtime and costs tens of
// microseconds more per read).
struct PinnedSlot {
  void *p = nullptr;
  ~PinnedSlot() {
    if (p) (void)hipHostFree(p);
  }
};

void *pinned_slot() {
  thread_local PinnedSlot slot;
  if (!slot.p) AMG_HIP(hipHostMalloc(&slot.p, 64, hipHostMallocDefault));
  return slot.p;
}

// Copy `bytes` (<= 64) from device memory to `dst` on the host; synchronises s.
void read_small(void *dst, const void *dptr, size_t bytes, hipStream_t s) {
  void *h = pinned_slot();
  AMG_HIP(hipMemcpyAsync(h, dptr, bytes, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  std::memcpy(dst, h, bytes);
}

int read_int(const int *dptr, hipStream_t s) {
  int v = 0;
  read_small(&v, dptr, sizeof(int), s);
  return v;
}

// ------------------------------------------------------------- validation
// flags[0]: malformed structure, flags[1]: a_ii <= 0 or missing diagonal,
// flags[2]: non-finite value, flags[3]: not bitwise symmetric.
__global__ void k_validate_rows(int n, int64_t nnz, const int *rp, const int *ci, const double *v,
                                int *flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == 0 && rp[0] != 0) atomicOr(&flags[0], 1);
  if (i == n - 1 && static_cast<int64_t>(rp[n]) != nnz) atomicOr(&flags[0], 1);
  const int lo = rp[i], hi = rp[i + 1];
  if (lo < 0 || hi < lo || static_cast<int64_t>(hi) > nnz) { atomicOr(&flags[0], 1); return; }
  bool diag = false;
  for (int k = lo; k < hi; ++k) {
    const int j = ci[k];
    if (j < 0 || j >= n || (k > lo && j <= ci[k - 1])) { atomicOr(&flags[0], 1); return; }
    const double a = v[k];
    if (!isfinite(a)) atomicOr(&flags[2], 1);
    if (j == i) {
      diag = true;
      if (!(a > 0.0)) atomicOr(&flags[1], 1);
    }
  }
  if (!diag) atomicOr(&flags[1], 1);
}

// Run only after k_validate_rows found a well-formed structure.
__global__ void k_validate_sym(int n, const int *rp, const int *ci, const double *v, int *flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = ci[k];
    int lo = rp[j], hi = rp[j + 1] - 1, pos = -1;
    while (lo <= hi) {
      int mid = (lo + hi) >> 1;
      int c = ci[mid];
      if (c == i) { pos = mid; break; }
      if (c < i) lo = mid + 1; else hi = mid - 1;
    }
    if (pos < 0 || __double_as_longlong(v[pos]) != __double_as_longlong(v[k])) {
      atomicOr(&flags[3], 1);
      return;
    }
  }
}

// ------------------------------------------------- diagonals and smoothing
__global__ void k_diag(int n, const int *rp, const int *ci, const double *v, double *d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k)
    if (ci[k] == i) a = v[k];
  d[i] = a;
}

// l1-Jacobi (Sec. 3.1): M_ii = sum_j |a_ij| folded in CSR order; dinv = 1/M_ii.
__global__ void k_l1_dinv(int n, const int *rp, const double *v, double *dinv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) m = m + fabs(v[k]);
  dinv[i] = 1.0 / m;
}

// binary32 diagonal of the mixed-precision V-cycle: the same fold over the
// values rounded to binary32, carried out in binary32.
__global__ void k_l1_dinv_f(int n, const int *rp, const double *v, float *dinv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float m = 0.0f;
  for (int k = rp[i]; k < rp[i + 1]; ++k) m = m + fabsf(static_cast<float>(v[k]));
  dinv[i] = 1.0f / m;
}

__global__ void k_fill(int n, double *x, double val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = val;
}

// max |x| by atomicMax on the IEEE bit pattern (order independent for
// x >= 0), one atomic per wavefront after a wavefront maximum.
__global__ void __launch_bounds__(kBlock) k_absmax(int n, const double *x, unsigned long long *out,
                                                   int *nonfinite) {
  unsigned long long m = 0;
  bool bad = false;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double a = fabs(x[i]);
    if (!isfinite(a)) bad = true;
    else m = max(m, static_cast<unsigned long long>(__double_as_longlong(a)));
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, static_cast<unsigned long long>(__shfl_xor(m, o, 64)));
  const unsigned long long anybad = __ballot(bad);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (m) atomicMax(out, m);
    if (anybad) atomicOr(nonfinite, 1);
  }
}

__global__ void k_scale_by_max(int n, double *x, const unsigned long long *mx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m = __longlong_as_double(static_cast<long long>(*mx));
  x[i] = (m > 0.0) ? x[i] / m : 1.0;
}

__global__ void k_check_finite(int n, const double *x, int *flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicOr(flag, 1);
}

// flag unless every entry is finite and positive (a usable learned vector)
__global__ void k_check_usable(int n, const double *x, int *flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(isfinite(x[i]) && x[i] > 0.0)) atomicOr(flag, 1);
}

// ------------------------------------------------------- matching weights
// w_hat = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2), evaluated with
// i = min(row, col) so both stored copies of an edge get the same bits:
// num = ((2 a) w_lo) w_hi, den = (a_lolo w_lo) w_lo + (a_hihi w_hi) w_hi.
// Eligible edges (a_ij != 0, w_hat > 0) keep their weight, others get -1.
// Decoupled aggregation (Sec. 4.1): with row-block bounds `off` (nparts + 1
// ascending offsets, off[0] = 0, off[nparts] = n) an edge is eligible only
// inside its row's block.
__global__ void k_weights(int n, const int *rp, const int *ci, const double *v, const double *d,
                          const double *w, double *wgt, const int *off, int nparts) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int blo = 0, bhi = n;   // columns of row i's block
  if (off) {
    int lo = 0, hi = nparts;   // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= i) lo = mid;
      else hi = mid;
    }
    blo = off[lo];
    bhi = off[lo + 1];
  }
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = ci[k];
    const double a = v[k];
    double out = -1.0;
    if (j != i && a != 0.0 && j >= blo && j < bhi) {
      const int lo = j < i ? j : i, hi = j < i ? i : j;
      const double wl = w[lo], wh = w[hi];
      const double num = ((2.0 * a) * wl) * wh;
      const double den = (d[lo] * wl) * wl + (d[hi] * wh) * wh;
      const double x = 1.0 - num / den;
      if (x > 0.0) out = x;
    }
    wgt[k] = out;
  }
}

// Row-block bounds of the coarse matrix of a pairwise step: the aggregate of
// a block's first row is the block's first coarse row (aggregates lie inside
// blocks and are numbered by their smallest row).
__global__ void k_coarse_offsets(int nparts, const int *off, int n, const int *agg, int nc,
                                 int *offc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > nparts) return;
  const int o = off[p];
  offc[p] = (o < n) ? agg[o] : nc;
}

// Strict total order on edges: weight, then max endpoint, then min endpoint.
__device__ __forceinline__ bool key_gt(double wa, int ha, int la, double wb, int hb, int lb) {
  if (wa != wb) return wa > wb;
  if (ha != hb) return ha > hb;
  return la > lb;
}

// Matching by locally dominant edges: every undecided vertex names its
// heaviest eligible edge to an undecided neighbour (its candidate); mutual
// choices are matched.  Under the strict total order this reproduces the
// sequential greedy matching (and Suitor's result) whatever the round
// structure.
//
// Rounds run on worklists.  A candidate stays the best choice until it is
// matched itself (the undecided set only shrinks), so after round 0 (all
// vertices) only the undecided neighbours that had named a newly matched
// vertex recompute their candidate, and a new mutual pair always contains
// such a vertex: round t = notify (matched list of t-1 -> recompute list,
// whose candidates are recomputed there), commit over the recompute list.  The
// state after every round equals that of all-vertex rounds; the matching
// ends when a recompute list is empty.  Lists are unordered (atomic
// appends); the result does not depend on their order.
//
// List kernels run grid-stride over a device-side count; list == nullptr
// means "every vertex 0..n-1".

// Heaviest eligible edge of i (row entries [b, e)) to an undecided
// neighbour, or -1.  Entries are taken eight at a time: their weights and
// columns, then the neighbours' states, are all in flight before any test
// (the maximum under the strict order does not depend on the scan order).
__device__ __forceinline__ int best_candidate_in(int i, int b, int e, const int *ci, const double *wgt,
                                                 const int *mate) {
  int best = -1, bh = 0, bl = 0;
  double bw = 0.0;
  for (int k0 = b; k0 < e; k0 += 8) {
    double x[8];
    int j[8], mj[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u < e ? k0 + u : e - 1;
      x[u] = wgt[k];
      j[u] = ci[k];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) mj[u] = mate[j[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u >= e || !(x[u] > 0.0) || mj[u] != kFree) continue;
      const int hi = j[u] > i ? j[u] : i, lo = j[u] > i ? i : j[u];
      if (best < 0 || key_gt(x[u], hi, lo, bw, bh, bl)) { best = j[u]; bw = x[u]; bh = hi; bl = lo; }
    }
  }
  return best;
}

// Heaviest eligible edge of i to an undecided neighbour (-1: none).
__device__ __forceinline__ int best_candidate(int i, const int *rp, const int *ci, const double *wgt,
                                              const int *mate) {
  return best_candidate_in(i, rp[i], rp[i + 1], ci, wgt, mate);
}

__global__ void __launch_bounds__(kBlock) k_mm_cand(int n, const int *rp, const int *ci,
                                                    const double *wgt, const int *mate,
                                                    int *cand) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (mate[i] == kFree) cand[i] = best_candidate(i, rp, ci, wgt, mate);
}

// Appends to the round lists are staged per workgroup in LDS and reserved
// in the global list with one atomic per workgroup pass (the lists are
// unordered); a full stage falls back to one atomic per entry.
constexpr int kStage = 1024;

// Mutual candidates are matched and appended to the matched list: both
// endpoints may be on the list, so the thread that claims the smaller
// endpoint (compare-and-swap from undecided) writes the pair, once.
// Vertices without a candidate become singletons.
__global__ void __launch_bounds__(kBlock) k_mm_commit(int n, const int *list, const int *cnt,
                                                      int *mate, const int *cand, int *mlist,
                                                      int *mcnt) {
  __shared__ int sbuf[kStage];
  __shared__ int scnt, sbase;
  const int m = list ? *cnt : n;
  for (int base = blockIdx.x * blockDim.x; base < m; base += gridDim.x * blockDim.x) {
    if (threadIdx.x == 0) scnt = 0;
    __syncthreads();
    const int q = base + threadIdx.x;
    if (q < m) {
      const int i = list ? list[q] : q;
      if (mate[i] == kFree) {
        const int c = cand[i];
        if (c < 0) {
          mate[i] = kSingle;
        } else if (cand[c] == i) {
          const int lo = c < i ? c : i, hi = c < i ? i : c;
          if (atomicCAS(&mate[lo], kFree, hi) == kFree) {
            mate[hi] = lo;
            const int pos = atomicAdd(&scnt, 2);
            if (pos + 1 < kStage) {
              sbuf[pos] = lo;
              sbuf[pos + 1] = hi;
            } else {
              const int g = atomicAdd(mcnt, 2);
              mlist[g] = lo;
              mlist[g + 1] = hi;
            }
          }
        }
      }
    }
    __syncthreads();
    const int c = min(scnt, kStage) & ~1;
    if (threadIdx.x == 0) sbase = c ? atomicAdd(mcnt, c) : 0;
    __syncthreads();
    for (int e = threadIdx.x; e < c; e += blockDim.x) mlist[sbase + e] = sbuf[e];
    __syncthreads();
  }
}

// Undecided neighbours whose candidate was just matched go on the recompute
// list, and the thread that lists u recomputes its candidate at once.  Each
// such u is found exactly once: its candidate is one vertex, which is on the
// matched list once (commit writes a pair once) and holds u once in its row;
// the new candidate is undecided (mate does not change in this kernel), so it
// never equals a matched vertex another thread compares against.  A team of
// kTeam lanes per matched vertex, lane l taking its row entries l, l + kTeam, ...
constexpr int kTeam = 8;

__global__ void __launch_bounds__(kBlock) k_mm_notify(const int *mlist, const int *mcnt,
                                                      const int *rp, const int *ci,
                                                      const double *wgt, const int *mate,
                                                      int *cand, int *rlist, int *rcnt) {
  __shared__ int sbuf[kStage];
  __shared__ int scnt, sbase;
  const int64_t total = static_cast<int64_t>(*mcnt) * kTeam;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * blockDim.x; base < total;
       base += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (threadIdx.x == 0) scnt = 0;
    __syncthreads();
    const int64_t g = base + threadIdx.x;
    if (g < total) {
      const int v = mlist[g / kTeam];
      const int l = static_cast<int>(g % kTeam);
      for (int k = rp[v] + l; k < rp[v + 1]; k += kTeam) {
        // the state of u and its row bounds are read together
        const int u = ci[k];
        const double wk = wgt[k];
        const int mu = mate[u], cu = cand[u], bu = rp[u], eu = rp[u + 1];
        if (u == v || !(wk > 0.0) || mu != kFree || cu != v) continue;
        cand[u] = best_candidate_in(u, bu, eu, ci, wgt, mate);
        const int pos = atomicAdd(&scnt, 1);
        if (pos < kStage) sbuf[pos] = u;
        else rlist[atomicAdd(rcnt, 1)] = u;
      }
    }
    __syncthreads();
    const int c = min(scnt, kStage);
    if (threadIdx.x == 0) sbase = c ? atomicAdd(rcnt, c) : 0;
    __syncthreads();
    for (int e = threadIdx.x; e < c; e += blockDim.x) rlist[sbase + e] = sbuf[e];
    __syncthreads();
  }
}

// Rounds whose matched list is short run in one workgroup: the notify and
// commit passes of the multi-workgroup kernels, with workgroup barriers in
// place of kernel boundaries (the waves of a workgroup share one L1, so
// their global writes are visible to each other after a barrier) and the
// lists in LDS (entries past kMTCap in the global lists).  It returns when
// the matching is complete (state[0] = 0), or hands the current matched
// list back (mlist, *mcnt; state[0] = 1) when it grows past kMTList or
// after kMTRounds rounds; state[1] = rounds run.
constexpr int kMTThreads = 1024;
constexpr int kMTCap = 4096;
constexpr int kMTList = 512;   // measured at 160^3: 2048 slower than the multi-workgroup rounds
constexpr int kMTRounds = 4096;

__global__ void __launch_bounds__(kMTThreads) k_mm_tail(const int *rp, const int *ci, const double *wgt,
                                                        int *mate, int *cand, int *mlist, int *mcnt,
                                                        int *rlist, int *state) {
  __shared__ int Ml[kMTCap], Rl[kMTCap];
  __shared__ int mc_s, rc_s;
  const int t = threadIdx.x, nt = blockDim.x;
  int m = *mcnt;
  for (int e = t; e < m && e < kMTCap; e += nt) Ml[e] = mlist[e];
  int r = 0, status = 1;
  while (r < kMTRounds) {
    if (t == 0) rc_s = 0;
    __syncthreads();
    // notify: undecided neighbours whose candidate was just matched
    const int64_t total = static_cast<int64_t>(m) * kTeam;
    for (int64_t g = t; g < total; g += nt) {
      const int idx = static_cast<int>(g / kTeam), l = static_cast<int>(g % kTeam);
      const int v = idx < kMTCap ? Ml[idx] : mlist[idx];
      for (int k = rp[v] + l; k < rp[v + 1]; k += kTeam) {
        const int u = ci[k];
        const double wk = wgt[k];
        const int mu = mate[u], cu = cand[u], bu = rp[u], eu = rp[u + 1];
        if (u == v || !(wk > 0.0) || mu != kFree || cu != v) continue;
        cand[u] = best_candidate_in(u, bu, eu, ci, wgt, mate);
        const int pos = atomicAdd(&rc_s, 1);
        if (pos < kMTCap) Rl[pos] = u;
        else rlist[pos] = u;
      }
    }
    __syncthreads();
    const int rc = rc_s;
    ++r;
    if (rc == 0) {
      status = 0;
      break;
    }
    if (t == 0) mc_s = 0;
    __syncthreads();
    // commit: mutual candidates matched, vertices without one single
    for (int q = t; q < rc; q += nt) {
      const int i = q < kMTCap ? Rl[q] : rlist[q];
      if (mate[i] != kFree) continue;
      const int c = cand[i];
      if (c < 0) {
        mate[i] = kSingle;
      } else if (cand[c] == i) {
        const int lo = c < i ? c : i, hi = c < i ? i : c;
        if (atomicCAS(&mate[lo], kFree, hi) == kFree) {
          mate[hi] = lo;
          const int pos = atomicAdd(&mc_s, 2);
          if (pos < kMTCap) Ml[pos] = lo;
          else mlist[pos] = lo;
          if (pos + 1 < kMTCap) Ml[pos + 1] = hi;
          else mlist[pos + 1] = hi;
        }
      }
    }
    __syncthreads();
    m = mc_s;
    if (m > kMTList) break;
  }
  if (status != 0) {
    for (int e = t; e < m && e < kMTCap; e += nt) mlist[e] = Ml[e];
    if (t == 0) *mcnt = m;
  }
  if (t == 0) {
    state[0] = status;
    state[1] = r;
  }
}

// ------------------------------------------------------------ aggregation
// Aggregates are numbered by their smallest fine index, ascending.
__global__ void k_agg_flags(int n, const int *mate, int *flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = mate[i];
  flag[i] = (m < 0 || m > i) ? 1 : 0;
}

__global__ void k_agg_ids(int n, const int *mate, const int *pos, int *agg, int *rep) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = mate[i];
  const int root = (m >= 0 && m < i) ? m : i;
  agg[i] = pos[root];
  if (root == i) rep[pos[i]] = i;
}

// p_i = w_i / sqrt(w_lo^2 + w_hi^2) on a pair, w_i / |w_i| (1 if w_i = 0) on a singleton.
__global__ void k_pair_pvals(int n, const int *mate, const double *w, double *p) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = mate[i];
  const double wi = w[i];
  if (j < 0) { p[i] = (wi == 0.0) ? 1.0 : wi / fabs(wi); return; }
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  const double wl = w[lo], wh = w[hi];
  const double nrm = sqrt(wl * wl + wh * wh);
  p[i] = wi / nrm;
}

// w_c = P^T w, members ascending: rep first, then its mate.
__global__ void k_pair_restrict_w(int nc, const int *rep, const int *mate, const double *p,
                                  const double *w, double *wc) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int lo = rep[I], hi = mate[lo];
  double s = 0.0;
  s = s + p[lo] * w[lo];
  if (hi >= 0) s = s + p[hi] * w[hi];
  wc[I] = s;
}

// ------------------------------------------------------ Galerkin product
// A_c(I,J) = sum of (p_i p_j) a_ij over stored a_ij with agg(i) = I,
// agg(j) = J.  Terms of one coarse entry are folded in ascending (u, v),
// u = the fine index on the side of min(I,J), v = the other, so entries
// (I,J) and (J,I) fold identical term sequences (bitwise-symmetric A_c).
// Within one coarse row a term's position in that order is the 64-bit key
// (J << 32) | k32, J = agg(j) for the fine entry a_ij, i = member m of the
// pair (0 = lo, 1 = hi): for J >= I, u = i and v = j, so the lo terms come
// first, each member's by j, and k32 = m * 2^31 + j; for J < I, u = j and
// v = i, so k32 = 2 j + m.  Keys of one row are distinct (a fine row holds a
// column once).
__device__ __forceinline__ unsigned long long rap_key(int I, int J, int j, int m) {
  const unsigned k32 = (I <= J) ? ((static_cast<unsigned>(m) << 31) | static_cast<unsigned>(j))
                                : ((static_cast<unsigned>(j) << 1) | static_cast<unsigned>(m));
  return (static_cast<unsigned long long>(static_cast<unsigned>(J)) << 32) | k32;
}

// Rows wider than the wavefront sort takes: one thread inserts the row's
// terms into key order in (tK, tT) at toff[I], then folds the runs of equal J
// in place, leaving the row's entries in (tJ, tT) from toff[I] on.
constexpr int kRapWaveMax = 512;

__global__ void __launch_bounds__(kBlock) k_rap_terms(int nc, const int *rep, const int *mate,
                                                      const int *rp, const int *ci, const double *v,
                                                      const int *agg, const double *p,
                                                      const int *toff, int *tJ,
                                                      unsigned long long *tK, double *tT,
                                                      int *ucnt) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int base = toff[I], c = toff[I + 1] - base;
  if (c <= kRapWaveMax) return;   // register or wavefront sort
  const int lo = rep[I], hi = mate[lo];
  int q = 0;
  for (int m = 0; m < 2; ++m) {
    const int i = (m == 0) ? lo : hi;
    if (i < 0) break;
    const double pi = p[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int j = ci[k];
      const unsigned long long key = rap_key(I, agg[j], j, m);
      const double t = (pi * p[j]) * v[k];
      int r = q;
      while (r > 0 && key < tK[base + r - 1]) {
        tK[base + r] = tK[base + r - 1];
        tT[base + r] = tT[base + r - 1];
        --r;
      }
      tK[base + r] = key;
      tT[base + r] = t;
      ++q;
    }
  }
  // runs of equal J, each folded from its first term; the u-th run's entry
  // overwrites slot u, which no later run reads
  int u = 0;
  for (int r = 0; r < c;) {
    const unsigned J = static_cast<unsigned>(tK[base + r] >> 32);
    double sum = tT[base + r];
    int e = r + 1;
    while (e < c && static_cast<unsigned>(tK[base + e] >> 32) == J) { sum = sum + tT[base + e]; ++e; }
    tJ[base + u] = static_cast<int>(J);
    tT[base + u] = sum;
    ++u;
    r = e;
  }
  ucnt[I] = u;
}

// Rows of kRapReg < c <= kRapWaveMax terms: one wavefront per coarse row.
// The terms go to LDS under their keys, padded to a power of two with keys
// that sort last; a bitonic network sorts them; the lane holding a run's
// first term folds the run in order and writes it to (tJ, tT) at toff[I] +
// the run's rank (a ballot prefix count).
__global__ void __launch_bounds__(kWave) k_rap_wave(int nc, const int *__restrict__ rep,
                                                    const int *__restrict__ mate,
                                                    const int *__restrict__ rp,
                                                    const int *__restrict__ ci,
                                                    const double *__restrict__ v,
                                                    const int *__restrict__ agg,
                                                    const double *__restrict__ p,
                                                    const int *__restrict__ toff,
                                                    int *__restrict__ tJ, double *__restrict__ tT,
                                                    int *__restrict__ ucnt) {
  __shared__ unsigned long long sk[kRapWaveMax];
  __shared__ double st[kRapWaveMax];
  const int lane = threadIdx.x;
  for (int I = blockIdx.x; I < nc; I += gridDim.x) {   // uniform in the workgroup
    const int base = toff[I], c = toff[I + 1] - base;
    if (c == 0 || c > kRapWaveMax) continue;
    const int lo = rep[I], hi = mate[lo];
    const int b0 = rp[lo], n0 = rp[lo + 1] - b0;
    const int b1 = hi >= 0 ? rp[hi] : 0;
    const double plo = p[lo], phi = hi >= 0 ? p[hi] : 0.0;
    int P = kWave / 2;
    while (P < c) P <<= 1;
    for (int q = lane; q < P; q += kWave) {
      unsigned long long key = ~0ull;
      double t = 0.0;
      if (q < c) {
        const int m = q < n0 ? 0 : 1;
        const int e = m ? b1 + (q - n0) : b0 + q;
        const int j = ci[e];
        key = rap_key(I, agg[j], j, m);
        t = ((m ? phi : plo) * p[j]) * v[e];
      }
      sk[q] = key;
      st[q] = t;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int t = lane; t < (P >> 1); t += kWave) {
          const int a = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
          const int bq = a + jj;
          const unsigned long long ka = sk[a], kb = sk[bq];
          const bool sw = ((a & k) == 0) ? (kb < ka) : (ka < kb);
          if (sw) {
            const double ta = st[a], tb = st[bq];
            sk[a] = kb;
            sk[bq] = ka;
            st[a] = tb;
            st[bq] = ta;
          }
        }
        __syncthreads();
      }
    }
    int done = 0;
    for (int q0 = 0; q0 < c; q0 += kWave) {
      const int q = q0 + lane;
      const unsigned J = q < c ? static_cast<unsigned>(sk[q] >> 32) : 0u;
      const bool head = q < c && (q == 0 || static_cast<unsigned>(sk[q - 1] >> 32) != J);
      const unsigned long long mask = __ballot(head);
      if (head) {
        double sum = st[q];
        for (int r = q + 1; r < c && static_cast<unsigned>(sk[r] >> 32) == J; ++r) sum = sum + st[r];
        const int rank = done + __popcll(mask & ((1ull << lane) - 1ull));
        tJ[base + rank] = static_cast<int>(J);
        tT[base + rank] = sum;
      }
      done += __popcll(mask);
    }
    if (lane == 0) ucnt[I] = done;
    __syncthreads();   // the next row overwrites sk, st
  }
}

// Coarse rows whose pair has at most kRapReg terms (the common case) sort
// and fold their terms in registers: gather, a bitonic network on the
// (J, key) order, then the runs of equal J folded from their first term --
// the order and the fold of the wide-row kernels.  The row's entries go
// to slots [I * kRapReg, I * kRapReg + ucnt[I]) of (uJ, uV) and are copied
// to their CSR place once the row lengths are scanned (k_rap_place).  Wider
// rows get tcnt = their term count and take the wavefront sort (k_rap_wave)
// or, past kRapWaveMax terms, the one-thread sort (k_rap_terms); narrow
// rows get tcnt = 0.
constexpr int kRapReg = 16;

// Compile-time loop: f(integral_constant<int, i>) for i = 0 .. N-1, so that
// register arrays are only ever indexed by constants.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__global__ void __launch_bounds__(kBlock) k_rap_reg(int nc, const int *__restrict__ rep,
                                                    const int *__restrict__ mate,
                                                    const int *__restrict__ rp,
                                                    const int *__restrict__ ci,
                                                    const double *__restrict__ v,
                                                    const int *__restrict__ agg,
                                                    const double *__restrict__ p,
                                                    int *__restrict__ tcnt, int *__restrict__ ucnt,
                                                    int *__restrict__ uJ, double *__restrict__ uV) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int lo = rep[I], hi = mate[lo];
  const int b0 = rp[lo], n0 = rp[lo + 1] - b0;
  const int b1 = hi >= 0 ? rp[hi] : 0, n1 = hi >= 0 ? rp[hi + 1] - b1 : 0;
  const int c = n0 + n1;
  if (c > kRapReg) {
    tcnt[I] = c;
    return;
  }
  int J[kRapReg];
  unsigned long long K[kRapReg];
  double T[kRapReg];
  static_for<kRapReg>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    J[q] = INT_MAX;
    K[q] = ~0ull;
    T[q] = 0.0;
    if (q < c) {
      const int i = q < n0 ? lo : hi;
      const int e = q < n0 ? b0 + q : b1 + (q - n0);
      const int j = ci[e];
      const int Jq = agg[j];
      const unsigned u = static_cast<unsigned>(I <= Jq ? i : j);
      const unsigned w2 = static_cast<unsigned>(I <= Jq ? j : i);
      J[q] = Jq;
      K[q] = (static_cast<unsigned long long>(u) << 32) | w2;
      T[q] = (p[i] * p[j]) * v[e];
    }
  });
  // bitonic sort, ascending by (J, K); padding (INT_MAX, ~0) sorts last.
  // Stages (k, j) = (2,1) (4,2) (4,1) (8,4) (8,2) (8,1) (16,8) (16,4) (16,2) (16,1).
  static_assert(kRapReg == 16, "the stage table below is for 16 slots");
  static_for<10>([&](auto st) {
    constexpr int kk[10] = {2, 4, 4, 8, 8, 8, 16, 16, 16, 16};
    constexpr int jv[10] = {1, 2, 1, 4, 2, 1, 8, 4, 2, 1};
    constexpr int k = kk[decltype(st)::value], jj = jv[decltype(st)::value];
    static_for<kRapReg>([&](auto ai) {
      constexpr int a = decltype(ai)::value, bb = a ^ jj;
      if constexpr (bb > a) {
        const bool lt = J[bb] < J[a] || (J[bb] == J[a] && K[bb] < K[a]);   // (b) < (a)
        const bool gt = J[a] < J[bb] || (J[a] == J[bb] && K[a] < K[bb]);   // (a) < (b)
        const bool sw = ((a & k) == 0) ? lt : gt;
        const int ja = J[a], jb = J[bb];
        const unsigned long long ka = K[a], kb = K[bb];
        const double ta = T[a], tb = T[bb];
        J[a] = sw ? jb : ja;
        J[bb] = sw ? ja : jb;
        K[a] = sw ? kb : ka;
        K[bb] = sw ? ka : kb;
        T[a] = sw ? tb : ta;
        T[bb] = sw ? ta : tb;
      }
    });
  });
  // runs of equal J: T[q] becomes the run's partial sum (started from its
  // first term); a run's last slot is an output
  int u = 0;
  const int64_t base = static_cast<int64_t>(I) * kRapReg;
  static_for<kRapReg>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    if (q < c) {
      if constexpr (q > 0)
        if (J[q] == J[q - 1]) T[q] = T[q - 1] + T[q];
      bool end = (q + 1 == c);
      if constexpr (q + 1 < kRapReg) end = end || (J[q + 1] != J[q]);
      if (end) {
        uJ[base + u] = J[q];
        uV[base + u] = T[q];
        ++u;
      }
    }
  });
  tcnt[I] = 0;
  ucnt[I] = u;
}

// Entries of narrow rows from slots I * kRapReg of (uJ, uV), of wide rows
// from toff[I] of (tJ, tT), to their CSR place.
__global__ void k_rap_place(int nc, const int *__restrict__ toff, const int *__restrict__ uJ,
                            const double *__restrict__ uV, const int *__restrict__ tJ,
                            const double *__restrict__ tT, const int *__restrict__ crp,
                            int *__restrict__ cci, double *__restrict__ cv) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const bool wide = toff[I] != toff[I + 1];
  const int64_t base = wide ? static_cast<int64_t>(toff[I]) : static_cast<int64_t>(I) * kRapReg;
  const int *sJ = wide ? tJ : uJ;
  const double *sV = wide ? tT : uV;
  const int b = crp[I], e = crp[I + 1];
  for (int q = 0; q < e - b; ++q) {
    cci[b + q] = sJ[base + q];
    cv[b + q] = sV[base + q];
  }
}

// Composite prolongator: agg <- agg_t(agg), p <- p * p_t(agg)  (left to right).
__global__ void k_compose(int n, int *agg, double *p, const int *agg_t, const double *p_t) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = agg[i];
  p[i] = p[i] * p_t[a];
  agg[i] = agg_t[a];
}

__global__ void k_iota(int n, int *a, double *p) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  a[i] = i;
  p[i] = 1.0;
}

// Members of each aggregate (CSR of P^T), ascending.
__global__ void k_count_members(int n, const int *agg, int *cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[agg[i]], 1);
}

__global__ void k_place_members(int n, const int *agg, const int *mptr, int *fill, int *mem) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = agg[i];
  const int pos = mptr[a] + atomicAdd(&fill[a], 1);
  mem[pos] = i;
}

__global__ void k_sort_members(int nc, const int *mptr, int *mem) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int b = mptr[I], e = mptr[I + 1];
  for (int q = b + 1; q < e; ++q) {
    const int x = mem[q];
    int r = q;
    while (r > b && mem[r - 1] > x) { mem[r] = mem[r - 1]; --r; }
    mem[r] = x;
  }
}

// ------------------------------------------------------------------ SELL
// Slots of each slice (64 x its widest row), and their total in 64 bits:
// the slot offsets are int32, so the host refuses a level whose total does
// not fit before any slot is indexed.
// Slots per slice (64 x the widest row), their total in total[0], and the
// widest and narrowest slice as total[1] = max width, total[2] = max of
// (2^31 - 1 - width).
__global__ void k_sell_width(int n, int nslices, const int *rp, int *slots, unsigned long long *total) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = 0, wmax = 0, wneg = 0;
  if (s < nslices) {
    int w = 0;
    const int r0 = s * kSlice, r1 = min(n, r0 + kSlice);
    for (int r = r0; r < r1; ++r) w = max(w, rp[r + 1] - rp[r]);
    v = static_cast<unsigned long long>(w) * kSlice;
    slots[s] = static_cast<int>(v);   // used only when the total fits
    wmax = static_cast<unsigned long long>(w);
    wneg = static_cast<unsigned long long>(0x7fffffff - w);
  }
  for (int o = 32; o > 0; o >>= 1) {   // every lane of the wavefront
    v += __shfl_xor(v, o, 64);
    wmax = max(wmax, static_cast<unsigned long long>(__shfl_xor(wmax, o, 64)));
    wneg = max(wneg, static_cast<unsigned long long>(__shfl_xor(wneg, o, 64)));
  }
  if ((threadIdx.x & 63) == 0) {
    if (v) atomicAdd(total, v);
    if (wmax) atomicMax(total + 1, wmax);
    if (wneg) atomicMax(total + 2, wneg);
  }
}

__global__ void k_sell_fill(int n, int nslices, const int *rp, const int *ci, const double *v,
                            const int *sptr, int *scol, double *sval) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nslices * kSlice) return;
  const int s = r / kSlice, lane = r % kSlice;
  const int width = (sptr[s + 1] - sptr[s]) / kSlice;
  const int base = sptr[s] + lane;
  const int len = (r < n) ? rp[r + 1] - rp[r] : 0;
  const int start = (r < n) ? rp[r] : 0;
  const int pad_col = (r < n) ? r : n - 1;
  for (int k = 0; k < width; ++k) {
    if (k < len) {
      scol[base + k * kSlice] = ci[start + k];
      sval[base + k * kSlice] = v[start + k];
    } else {
      scol[base + k * kSlice] = pad_col;
      sval[base + k * kSlice] = 0.0;
    }
  }
}

// One wavefront per slice: base and 16-bit offsets of every slot group, or
// cbase = -1 for the whole slice when some group spans more than 16 bits.
// Counts the matrix entries (row lengths) and groups of compact slices.
__device__ __forceinline__ int wave_min_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ void __launch_bounds__(kBlock) k_sell_compact(int n, int nslices, const int *rp,
                                                         const int *sptr, const int *qptr,
                                                         const int *scol, int *cbase,
                                                         unsigned short *cdel,
                                                         unsigned long long *count) {
  const int s = blockIdx.x * (kBlock / kWave) + static_cast<int>(threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (s >= nslices) return;   // whole wavefront
  const int b = sptr[s], width = (sptr[s + 1] - b) / kSlice;
  const int64_t q0 = static_cast<int64_t>(qptr[s]) * kSlice;
  bool fits = true;
  for (int k = 0; k < width; ++k) {
    const int c = scol[b + k * kSlice + lane];
    fits = fits && (wave_max_i(c) - wave_min_i(c) <= 65535);
  }
  for (int k = 0; k < 4 * (qptr[s + 1] - qptr[s]); ++k) {
    const int64_t at = ((q0 + (k >> 2) * kSlice) + lane) * 4 + (k & 3);
    if (k >= width) {
      cdel[at] = 0;
      continue;
    }
    const int c = scol[b + k * kSlice + lane];
    const int mn = wave_min_i(c);
    cdel[at] = fits ? static_cast<unsigned short>(c - mn) : 0;
    if (lane == 0) cbase[b / kSlice + k] = fits ? mn : -1;
  }
  if (lane == 0 && fits) {
    const int r0 = s * kSlice, r1 = min(n, r0 + kSlice);
    atomicAdd(&count[0], static_cast<unsigned long long>(rp[r1] - rp[r0]));
    atomicAdd(&count[1], static_cast<unsigned long long>(width));
  }
}

__global__ void k_sell_quads(int nslices, const int *sptr, int *quads) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nslices) quads[s] = ((sptr[s + 1] - sptr[s]) / kSlice + 3) / 4;
}

__global__ void k_d2f(int64_t n, const double *a, float *b) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<float>(a[i]);
}

// ------------------------------------------------------- coarsest factor
__global__ void k_densify(int n, const int *rp, const int *ci, const double *v, double *D) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) D[static_cast<int64_t>(i) * n + ci[k]] = v[k];
}

// Right-looking Cholesky in one workgroup, in place on the row-major lower
// triangle.  Entry (i,l) receives the updates -L_ij L_lj for j = 0, 1, ...
// in ascending order, the same fold as the left-looking definition
// L_il = (a_il - sum_{j<l} L_ij L_lj) / L_ll.
// Right-looking Cholesky in one workgroup (n <= kDenseMax), in panels of
// kPanel columns: inside a panel, step j takes the pivot, scales column j
// (kept in LDS) and updates the panel's remaining columns; after the panel
// the trailing lower triangle receives the panel's kPanel updates, applied
// in column order, in one pass (a wavefront per row, lanes along the row).
// Entry (i, l) thus receives - L_ik L_lk for k = 0, 1, ... in order: the
// fold of the column-by-column definition.
constexpr int kPanel = 8;

__global__ void __launch_bounds__(1024) k_cholesky(int n, double *D, int *flag) {
  __shared__ int bad;
  __shared__ double col[kPanel][kDenseMax];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += kPanel) {
    const int j1 = min(n, j0 + kPanel);
    for (int j = j0; j < j1; ++j) {
      if (threadIdx.x == 0) {
        const double piv = D[static_cast<int64_t>(j) * n + j];
        if (!(piv > 0.0)) bad = 1;
        else D[static_cast<int64_t>(j) * n + j] = sqrt(piv);
      }
      __syncthreads();
      if (bad) break;
      const double ljj = D[static_cast<int64_t>(j) * n + j];
      double *cj = col[j - j0];
      for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) {
        const double v = D[static_cast<int64_t>(i) * n + j] / ljj;
        D[static_cast<int64_t>(i) * n + j] = v;
        cj[i] = v;
      }
      __syncthreads();
      // panel columns l in (j, j1): rows i >= l
      for (int t = threadIdx.x; t < (j1 - j - 1) * n; t += blockDim.x) {
        const int l = j + 1 + t / n, i = t % n;
        if (i >= l) D[static_cast<int64_t>(i) * n + l] = D[static_cast<int64_t>(i) * n + l] - cj[i] * cj[l];
      }
      __syncthreads();
    }
    if (bad) break;
    // trailing block: rows i >= j1, columns l in [j1, i]
    const int kb = j1 - j0;
    for (int i = j1 + wid; i < n; i += nw) {
      double *row = D + static_cast<int64_t>(i) * n;
      for (int l = j1 + lane; l <= i; l += kWave) {
        double x = row[l];
        for (int k = 0; k < kb; ++k) x = x - col[k][i] * col[k][l];
        row[l] = x;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && bad) *flag = 1;
}

// Inverse of the coarsest matrix from its Cholesky factor L (row-major lower
// triangle of D): thread j solves L y = e_j (k ascending), then L^T x = y
// (k descending) and stores x as column j of the column-major inverse.
// Columns of A^-1: lane jj (< kInvCols) of the one-wavefront workgroup
// solves L y = e_j (k ascending), then L^T x = y (k descending), j = 16 g + jj
// -- the fold order of the direct solve.  The 16 solution vectors live in LDS
// (entry k of column jj at Xs[k][jj]); the factor row needed at step i (row i
// of L forward, row i of L^T = Dt backward) is in LDS too, the next one
// loaded into registers by the whole wavefront during the current fold.
// Terms are read kB at a time ahead of the sequential fold.  The workgroup
// finally writes its columns to Ainv (column-major: column c at Ainv[c n ..]).
constexpr int kInvCols = 16;

template <bool kBack>
__device__ __forceinline__ void inv_fetch(const double *__restrict__ M, int n, int row, int lo,
                                          int hi, double (&pre)[kDenseMax / kWave]) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kDenseMax / kWave; ++q) {
    const int idx = q * kWave + lane;
    if (idx >= lo && idx <= hi) pre[q] = M[static_cast<int64_t>(row) * n + idx];
  }
}

__device__ __forceinline__ void inv_store(double *Lr, int lo, int hi,
                                          const double (&pre)[kDenseMax / kWave]) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kDenseMax / kWave; ++q) {
    const int idx = q * kWave + lane;
    if (idx >= lo && idx <= hi) Lr[idx] = pre[q];
  }
}

__global__ void __launch_bounds__(kWave) k_chol_inverse(int n, const double *__restrict__ D,
                                                        const double *__restrict__ Dt,
                                                        double *__restrict__ Ainv) {
  __shared__ double Xs[kDenseMax][kInvCols];
  __shared__ double Lr[2][kDenseMax];
  const int jj = threadIdx.x, j0 = blockIdx.x * kInvCols;
  const int j = j0 + jj;
  const bool act = jj < kInvCols && j < n;
  constexpr int kB = 32;
  double pre[kDenseMax / kWave];
  // forward: step i uses row i of L, entries 0..i
  inv_fetch<false>(D, n, 0, 0, 0, pre);
  inv_store(Lr[0], 0, 0, pre);
  __syncthreads();
  for (int i = 0; i < n; ++i) {
    const double *L = Lr[i & 1];
    if (i + 1 < n) inv_fetch<false>(D, n, i + 1, 0, i + 1, pre);
    if (act) {
      double s = (i == j) ? 1.0 : 0.0;
      int k = 0;
      for (; k + kB <= i; k += kB) {
        double a[kB], b[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          a[u] = L[k + u];
          b[u] = Xs[k + u][jj];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) s = s - a[u] * b[u];
      }
      for (; k < i; ++k) s = s - L[k] * Xs[k][jj];
      Xs[i][jj] = s / L[i];
    }
    if (i + 1 < n) inv_store(Lr[(i + 1) & 1], 0, i + 1, pre);
    __syncthreads();
  }
  // backward: step i uses row i of L^T (column i of L), entries i..n-1
  inv_fetch<true>(Dt, n, n - 1, n - 1, n - 1, pre);
  inv_store(Lr[(n - 1) & 1], n - 1, n - 1, pre);
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    const double *L = Lr[i & 1];
    if (i > 0) inv_fetch<true>(Dt, n, i - 1, i - 1, n - 1, pre);
    if (act) {
      double s = Xs[i][jj];
      int k = n - 1;
      for (; k - kB >= i; k -= kB) {
        double a[kB], b[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          a[u] = L[k - u];
          b[u] = Xs[k - u][jj];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) s = s - a[u] * b[u];
      }
      for (; k > i; --k) s = s - L[k] * Xs[k][jj];
      Xs[i][jj] = s / L[i];
    }
    if (i > 0) inv_store(Lr[(i - 1) & 1], i - 1, n - 1, pre);
    __syncthreads();
  }
  const int nc = min(kInvCols, n - j0);
  for (int t = threadIdx.x; t < nc * n; t += blockDim.x) {
    const int c = t / n, i = t % n;
    Ainv[static_cast<int64_t>(j0 + c) * n + i] = Xs[i][c];
  }
}

// out = in^T for an n x n row-major matrix.
__global__ void k_transpose_sq(int n, const double *__restrict__ in, double *__restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(n) * n) return;
  const int r = static_cast<int>(t / n), c = static_cast<int>(t % n);
  out[static_cast<int64_t>(c) * n + r] = in[t];
}

// --------------------------------------------------------- host helpers

double now_ms() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double, std::milli>(clk::now().time_since_epoch()).count();
}

void check_flags(const dvec<int> &flags, hipStream_t s) {
  int f[4] = {0, 0, 0, 0};
  read_small(f, flags.p, sizeof(f), s);
  if (f[0]) fail(AMG_ERR_INVALID, "malformed CSR (row_ptr, column range or ordering)");
  if (f[2]) fail(AMG_ERR_NONFINITE, "non-finite matrix value");
  if (f[1]) fail(AMG_ERR_NOT_SPD, "missing or non-positive diagonal entry");
  if (f[3]) fail(AMG_ERR_INVALID, "matrix is not bitwise symmetric");
}

// ----------------------------------------------------- coded SELL values
// Distinct bit patterns of the slot values go into an open-addressing table
// of kDictSlots keys (linear probing; kDictEmpty, a signalling-NaN pattern
// that arithmetic never produces, marks a free slot).  count > kDictMax
// means "too many": the level stays plain.
constexpr int kDictSlots = 1024;
constexpr unsigned long long kDictEmpty = 0x7ff4a5a5a5a5a5a5ull;

__device__ __forceinline__ unsigned dict_hash(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  return static_cast<unsigned>(k) & (kDictSlots - 1);
}

// Probes are bounded: a key that does not find its place within kDictProbe
// slots marks the level as too varied (count > kDictMax), so no probe ever
// walks a crowded table.
constexpr int kDictProbe = 64;

__device__ __forceinline__ int dict_count(const int *count) {
  return __hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Slot of key k in the table, or -1 (absent).
__device__ __forceinline__ int dict_find(const unsigned long long *tab, unsigned long long k) {
  unsigned h = dict_hash(k);
  for (int probe = 0; probe < kDictProbe; ++probe) {
    const unsigned long long t = tab[h];
    if (t == k) return static_cast<int>(h);
    if (t == kDictEmpty) return -1;
    h = (h + 1) & (kDictSlots - 1);
  }
  return -1;
}

// Inserts k unless present; counts new keys.  Does nothing once the count
// has passed kDictMax (the level stays plain then).
__device__ __forceinline__ void dict_insert(unsigned long long *tab, int *count, unsigned long long k) {
  if (dict_count(count) > kDictMax) return;
  unsigned h = dict_hash(k);
  for (int probe = 0; probe < kDictProbe; ++probe) {
    unsigned long long t = tab[h];   // plain read first: present keys cost no atomic
    if (t == k) return;
    if (t == kDictEmpty) {
      t = atomicCAS(&tab[h], kDictEmpty, k);
      if (t == kDictEmpty) {
        atomicAdd(count, 1);
        return;
      }
      if (t == k) return;
    }
    h = (h + 1) & (kDictSlots - 1);
  }
  atomicAdd(count, kDictSlots);   // no place within the probe bound
}

// One wavefront removes duplicates among its 64 values before touching the
// table: the first lane still holding an unseen key inserts it for every
// lane with the same key.
__global__ void __launch_bounds__(kBlock) k_dict_insert(int64_t m, const double *__restrict__ v,
                                                        unsigned long long *tab, int *count) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
       i - lane < m; i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const unsigned long long k = i < m ? static_cast<unsigned long long>(__double_as_longlong(v[i])) : 0ull;
    bool pending = i < m;
    for (int it = 0;; ++it) {
      if ((it & 7) == 0 && __shfl(dict_count(count), 0) > kDictMax) return;   // wavefront-uniform
      const unsigned long long ball = __ballot(pending);
      if (ball == 0) break;
      const int leader = __ffsll(ball) - 1;
      const unsigned long long lk = __shfl(k, leader);
      if (lane == leader) dict_insert(tab, count, lk);
      if (pending && k == lk) pending = false;
    }
  }
}

// One workgroup: the occupied keys ranked by bit pattern (rank = number of
// smaller keys), rank[slot] for the encoder, dict[rank] = the value.
__global__ void __launch_bounds__(kBlock) k_dict_rank(const unsigned long long *tab, int *rank,
                                                      double *dict, float *dictf) {
  __shared__ unsigned long long keys[kDictSlots];
  for (int h = threadIdx.x; h < kDictSlots; h += blockDim.x) keys[h] = tab[h];
  __syncthreads();
  for (int h = threadIdx.x; h < kDictSlots; h += blockDim.x) {
    const unsigned long long k = keys[h];
    if (k == kDictEmpty) {
      rank[h] = -1;
      continue;
    }
    int r = 0;
    for (int q = 0; q < kDictSlots; ++q) r += (keys[q] != kDictEmpty && keys[q] < k) ? 1 : 0;
    rank[h] = r;
    const double x = __longlong_as_double(static_cast<long long>(k));
    dict[r] = x;
    if (dictf) dictf[r] = static_cast<float>(x);
  }
}

// One wavefront per slice: the code of every slot, stored by quads (padding 0).
__global__ void __launch_bounds__(kBlock) k_dict_encode(int nslices, const int *__restrict__ sptr,
                                                        const int *__restrict__ qptr,
                                                        const double *__restrict__ v,
                                                        const unsigned long long *__restrict__ tab,
                                                        const int *__restrict__ rank,
                                                        unsigned char *__restrict__ code) {
  const int s = blockIdx.x * (kBlock / kWave) + static_cast<int>(threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (s >= nslices) return;
  const int b = sptr[s], width = (sptr[s + 1] - b) / kSlice;
  const int64_t q0 = static_cast<int64_t>(qptr[s]) * kSlice;
  for (int k = 0; k < 4 * (qptr[s + 1] - qptr[s]); ++k) {
    int c = 0;
    if (k < width) {   // every slot value was inserted
      const int h = dict_find(tab, static_cast<unsigned long long>(__double_as_longlong(v[b + k * kSlice + lane])));
      c = h >= 0 ? rank[h] : 0;
    }
    code[((q0 + (k >> 2) * kSlice) + lane) * 4 + (k & 3)] = static_cast<unsigned char>(c);
  }
}

__global__ void k_fill_u64(int n, unsigned long long *a, unsigned long long x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = x;
}

// Table of the slot values of S (padding included) and their codes, when
// there are at most kDictMax distinct bit patterns.
void build_codes(Sell &S, hipStream_t s, bool want_float) {
  S.ndict = 0;
  if (S.nslots == 0) return;
  tvec<unsigned long long> tab(kDictSlots, s);
  tvec<int> cnt(1, s), rank(kDictSlots, s);
  hipLaunchKernelGGL(k_fill_u64, dim3(kDictSlots / kBlock), dim3(kBlock), 0, s, kDictSlots, tab.p,
                     kDictEmpty);
  AMG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int), s));
  const unsigned gi = static_cast<unsigned>(std::min<int64_t>(4096, ceil_div(S.nslots, kBlock)));
  hipLaunchKernelGGL(k_dict_insert, dim3(gi), dim3(kBlock), 0, s, S.nslots, S.val.p, tab.p, cnt.p);
  AMG_LAUNCH_CHECK();
  const int nd = read_int(cnt.p, s);
  if (nd < 1 || nd > kDictMax) return;
  S.dict.alloc(nd);
  if (want_float) S.dictf.alloc(nd);
  S.code.alloc(S.nquads * kSlice * 4);
  hipLaunchKernelGGL(k_dict_rank, dim3(1), dim3(kBlock), 0, s, tab.p, rank.p, S.dict.p,
                     want_float ? S.dictf.p : nullptr);
  hipLaunchKernelGGL(k_dict_encode, grid_for(static_cast<int64_t>(S.nslices) * kWave), dim3(kBlock), 0, s,
                     S.nslices, S.sptr.p, S.qptr.p, S.val.p, tab.p, rank.p, S.code.p);
  AMG_LAUNCH_CHECK();
  S.ndict = nd;
}

// code[i] = rank of v[i] in the table (every value was inserted)
__global__ void k_dict_encode_flat(int n, const double *__restrict__ v, const unsigned long long *__restrict__ tab,
                                   const int *__restrict__ rank, unsigned char *__restrict__ code) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int h = dict_find(tab, static_cast<unsigned long long>(__double_as_longlong(v[i])));
  code[i] = static_cast<unsigned char>(h >= 0 ? rank[h] : 0);
}

// P values of a level as codes into a table of their distinct bit patterns,
// when there are at most kDictMax of them (the binary64 prolongation and
// restriction then read one byte per row instead of eight).
void build_pcodes(Level &Lv, hipStream_t s) {
  Lv.npdict = 0;
  const int n = Lv.A.n;
  if (n <= 0 || !Lv.pval.p) return;
  tvec<unsigned long long> tab(kDictSlots, s);
  tvec<int> cnt(1, s), rank(kDictSlots, s);
  hipLaunchKernelGGL(k_fill_u64, dim3(kDictSlots / kBlock), dim3(kBlock), 0, s, kDictSlots, tab.p,
                     kDictEmpty);
  AMG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int), s));
  const unsigned gi = static_cast<unsigned>(std::min<int64_t>(4096, ceil_div(n, kBlock)));
  hipLaunchKernelGGL(k_dict_insert, dim3(gi), dim3(kBlock), 0, s, static_cast<int64_t>(n), Lv.pval.p, tab.p,
                     cnt.p);
  AMG_LAUNCH_CHECK();
  const int nd = read_int(cnt.p, s);
  if (nd < 1 || nd > kDictMax) return;
  Lv.pdict.alloc(nd);
  Lv.pcode.alloc(n);
  hipLaunchKernelGGL(k_dict_rank, dim3(1), dim3(kBlock), 0, s, tab.p, rank.p, Lv.pdict.p, nullptr);
  hipLaunchKernelGGL(k_dict_encode_flat, grid_for(n), dim3(kBlock), 0, s, n, Lv.pval.p, tab.p, rank.p,
                     Lv.pcode.p);
  AMG_LAUNCH_CHECK();
  Lv.npdict = nd;
}

void build_sell(Level &Lv, hipStream_t s, bool want_float, bool want_codes) {
  Sell &S = Lv.S;
  const int n = Lv.A.n;
  S.n = n;
  S.nslices = ceil_div(n, kSlice);
  tvec<int> slots(S.nslices, s);
  tvec<unsigned long long> total(3, s);
  S.sptr.alloc(S.nslices + 1);
  AMG_HIP(hipMemsetAsync(total.p, 0, 3 * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_sell_width, grid_for(S.nslices), dim3(kBlock), 0, s, n, S.nslices,
                     Lv.A.rp.p, slots.p, total.p);
  AMG_LAUNCH_CHECK();
  unsigned long long tw[3] = {0, 0, 0};
  read_small(tw, total.p, sizeof(tw), s);
  const unsigned long long nslots = tw[0];
  S.wmax = static_cast<int>(tw[1]);
  S.wmin = 0x7fffffff - static_cast<int>(tw[2]);
  if (nslots >= (1ull << 31))
    fail(AMG_ERR_UNSUPPORTED, "a level's SELL form needs 2^31 or more slots (rows of very different "
                              "lengths share slices); slot offsets are int32");
  exclusive_scan(slots.p, S.sptr.p, S.nslices, s);
  S.nslots = static_cast<int64_t>(nslots);
  S.col.alloc(S.nslots);
  S.val.alloc(S.nslots);
  hipLaunchKernelGGL(k_sell_fill, grid_for(static_cast<int64_t>(S.nslices) * kSlice), dim3(kBlock),
                     0, s, n, S.nslices, Lv.A.rp.p, Lv.A.ci.p, Lv.A.v.p, S.sptr.p, S.col.p, S.val.p);
  AMG_LAUNCH_CHECK();
  S.cbase.alloc(S.nslots / kSlice + kGroupPad);
  AMG_HIP(hipMemsetAsync(S.cbase.p + S.nslots / kSlice, 0, sizeof(int) * kGroupPad, s));
  S.qptr.alloc(S.nslices + 1);
  hipLaunchKernelGGL(k_sell_quads, grid_for(S.nslices), dim3(kBlock), 0, s, S.nslices, S.sptr.p, slots.p);
  AMG_LAUNCH_CHECK();
  exclusive_scan(slots.p, S.qptr.p, S.nslices, s);
  S.nquads = read_int(S.qptr.p + S.nslices, s);
  S.cdel.alloc(S.nquads * kSlice * 4);
  tvec<unsigned long long> cnt(2, s);
  AMG_HIP(hipMemsetAsync(cnt.p, 0, 2 * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_sell_compact, grid_for(static_cast<int64_t>(S.nslices) * kWave), dim3(kBlock),
                     0, s, n, S.nslices, Lv.A.rp.p, S.sptr.p, S.qptr.p, S.col.p, S.cbase.p, S.cdel.p,
                     cnt.p);
  AMG_LAUNCH_CHECK();
  unsigned long long hc[2];
  read_small(hc, cnt.p, sizeof(hc), s);
  S.nnz_compact = static_cast<int64_t>(hc[0]);
  S.groups_compact = static_cast<int64_t>(hc[1]);
  if (want_float) {
    S.valf.alloc(S.nslots);
    hipLaunchKernelGGL(k_d2f, grid_for(S.nslots), dim3(kBlock), 0, s, S.nslots, S.val.p, S.valf.p);
    AMG_LAUNCH_CHECK();
  }
  if (want_codes) build_codes(S, s, want_float);
}

// One pairwise step on (A, w): matching, aggregates, P values, w_c, A_c.
struct PairStep {
  int nc = 0;
  wsv<int> agg, rep, mate;     // carved from the setup workspace
  wsv<double> p;
  dvec<double> wc;             // these two become the next level
  DevCSR Ac;
  dvec<int> offc;              // row-block bounds of Ac (decoupled aggregation only)
};

// Workspace bytes of one pairwise step on (n rows, nnz entries): matching
// arrays, aggregation, the pair's outputs, the Galerkin staging (at most n
// coarse rows of kRapReg slots) and the general-path terms (at most nnz).
size_t pair_workspace_bytes(int64_t n, int64_t nnz) {
  return static_cast<size_t>(264 * n + 28 * nnz) + 64 * 256 + 4096;
}

// off: row-block bounds of A (nparts + 1 entries, device) for decoupled
// aggregation, or nullptr for one block.
void pairwise_step(const DevCSR &A, const double *w, const int *off, int nparts, hipStream_t s,
                   PairStep &out, Timing &tm, Arena &ws) {
  const int n = A.n;
  const dim3 g = grid_for(n), b(kBlock);
  double t0 = now_ms();
  ws.reserve(pair_workspace_bytes(n, A.nnz));
  wsv<double> d(ws, n), wgt(ws, A.nnz);
  hipLaunchKernelGGL(k_diag, g, b, 0, s, n, A.rp.p, A.ci.p, A.v.p, d.p);
  AMG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_weights, g, b, 0, s, n, A.rp.p, A.ci.p, A.v.p, d.p, w, wgt.p, off, nparts);
  AMG_LAUNCH_CHECK();
  out.mate = wsv<int>(ws, n);
  wsv<int> cand(ws, n), rlist(ws, n), mbuf0(ws, n), mbuf1(ws, n);
  int *mbuf[2] = {mbuf0.p, mbuf1.p};
  hipLaunchKernelGGL(k_fill_int, g, b, 0, s, n, out.mate.p, kFree);
  AMG_LAUNCH_CHECK();
  // Rounds are issued in batches of kBatch with one host read per batch.
  // cnt[2q] = matched-list length of the round before round q of the batch,
  // cnt[2q+1] = recompute-list length of round q.  Each vertex enters a
  // matched list once and a recompute list at most once per round, so n
  // entries bound every list; matched lists alternate between two buffers.
  const int kBatch = 16;   // even: round 0 of every batch reads mbuf[0]
  const dim3 gl(static_cast<unsigned>(std::min(1024, std::max(1, ceil_div(n, kBlock)))));
  wsv<int> cnt(ws, 2 * kBatch + 2);
  AMG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * (2 * kBatch + 2), s));
  hipLaunchKernelGGL(k_mm_cand, gl, b, 0, s, n, A.rp.p, A.ci.p, wgt.p, out.mate.p, cand.p);
  hipLaunchKernelGGL(k_mm_commit, gl, b, 0, s, n, nullptr, nullptr, out.mate.p, cand.p, mbuf[0],
                     cnt.p);
  AMG_LAUNCH_CHECK();
  int rounds = 1;
  for (;;) {
    // cnt[0] holds the matched-list length left by the previous round
    AMG_HIP(hipMemsetAsync(cnt.p + 1, 0, sizeof(int) * (2 * kBatch + 1), s));
    for (int q = 0; q < kBatch; ++q) {
      const int *mc = cnt.p + 2 * q;
      int *rc = cnt.p + 2 * q + 1;
      int *mc_next = cnt.p + 2 * q + 2;
      hipLaunchKernelGGL(k_mm_notify, gl, b, 0, s, mbuf[q % 2], mc, A.rp.p, A.ci.p, wgt.p,
                         out.mate.p, cand.p, rlist.p, rc);
      hipLaunchKernelGGL(k_mm_commit, gl, b, 0, s, n, rlist.p, rc, out.mate.p, cand.p,
                         mbuf[(q + 1) % 2], mc_next);
    }
    AMG_LAUNCH_CHECK();
    rounds += kBatch;
    int last[2];   // recompute-list length of the last round, matched-list length after it
    read_small(last, cnt.p + 2 * kBatch - 1, sizeof(last), s);
    if (last[0] == 0) break;
    if (rounds > n + 2 * kBatch) fail(AMG_ERR_DEVICE, "matching did not terminate");
    if (last[1] <= kMTList) {
      // the matched list (in mbuf[0]: kBatch is even) is short: continue in one workgroup
      hipLaunchKernelGGL(k_mm_tail, dim3(1), dim3(kMTThreads), 0, s, A.rp.p, A.ci.p, wgt.p,
                         out.mate.p, cand.p, mbuf[0], cnt.p + 2 * kBatch, rlist.p, cnt.p + 1);
      AMG_LAUNCH_CHECK();
      int st[2];
      read_small(st, cnt.p + 1, sizeof(st), s);
      rounds += st[1];
      if (st[0] == 0) break;
    }
    // carry the last matched-list length into cnt[0]
    AMG_HIP(hipMemcpyAsync(cnt.p, cnt.p + 2 * kBatch, sizeof(int), hipMemcpyDeviceToDevice, s));
  }
  tm.rounds += rounds;
  wsv<int> flag(ws, n), pos(ws, n + 1);
  hipLaunchKernelGGL(k_agg_flags, g, b, 0, s, n, out.mate.p, flag.p);
  AMG_LAUNCH_CHECK();
  exclusive_scan(flag.p, pos.p, n, s);
  const int nc = read_int(pos.p + n, s);
  out.nc = nc;
  out.agg = wsv<int>(ws, n);
  out.rep = wsv<int>(ws, nc);
  out.p = wsv<double>(ws, n);
  out.wc.alloc(nc);
  hipLaunchKernelGGL(k_agg_ids, g, b, 0, s, n, out.mate.p, pos.p, out.agg.p, out.rep.p);
  hipLaunchKernelGGL(k_pair_pvals, g, b, 0, s, n, out.mate.p, w, out.p.p);
  hipLaunchKernelGGL(k_pair_restrict_w, grid_for(nc), b, 0, s, nc, out.rep.p, out.mate.p, out.p.p,
                     w, out.wc.p);
  AMG_LAUNCH_CHECK();
  if (off) {
    out.offc.alloc(nparts + 1);
    hipLaunchKernelGGL(k_coarse_offsets, grid_for(nparts + 1), b, 0, s, nparts, off, n, out.agg.p, nc,
                       out.offc.p);
    AMG_LAUNCH_CHECK();
  }
  AMG_HIP(hipStreamSynchronize(s));
  double t1 = now_ms();
  tm.match_ms += t1 - t0;

  // Galerkin product
  const dim3 gc = grid_for(nc);
  wsv<int> tcnt(ws, nc), toff(ws, nc + 1), ucnt(ws, nc), uJ(ws, static_cast<size_t>(nc) * kRapReg);
  wsv<double> uV(ws, static_cast<size_t>(nc) * kRapReg);
  hipLaunchKernelGGL(k_rap_reg, gc, b, 0, s, nc, out.rep.p, out.mate.p, A.rp.p, A.ci.p, A.v.p,
                     out.agg.p, out.p.p, tcnt.p, ucnt.p, uJ.p, uV.p);
  AMG_LAUNCH_CHECK();
  exclusive_scan(tcnt.p, toff.p, nc, s);
  const int nterms = read_int(toff.p + nc, s);
  wsv<int> tJ(ws, nterms);
  wsv<unsigned long long> tK(ws, nterms);
  wsv<double> tT(ws, nterms);
  if (nterms > 0) {
    const unsigned gw = static_cast<unsigned>(std::min(nc, 1 << 20));
    hipLaunchKernelGGL(k_rap_wave, dim3(gw), dim3(kWave), 0, s, nc, out.rep.p,
                       out.mate.p, A.rp.p, A.ci.p, A.v.p, out.agg.p, out.p.p, toff.p, tJ.p, tT.p,
                       ucnt.p);
    hipLaunchKernelGGL(k_rap_terms, gc, b, 0, s, nc, out.rep.p, out.mate.p, A.rp.p, A.ci.p, A.v.p,
                       out.agg.p, out.p.p, toff.p, tJ.p, tK.p, tT.p, ucnt.p);
    AMG_LAUNCH_CHECK();
  }
  out.Ac.n = nc;
  out.Ac.rp.alloc(nc + 1);
  exclusive_scan(ucnt.p, out.Ac.rp.p, nc, s);
  out.Ac.nnz = read_int(out.Ac.rp.p + nc, s);
  out.Ac.ci.alloc(out.Ac.nnz);
  out.Ac.v.alloc(out.Ac.nnz);
  hipLaunchKernelGGL(k_rap_place, gc, b, 0, s, nc, toff.p, uJ.p, uV.p, tJ.p, tT.p, out.Ac.rp.p,
                     out.Ac.ci.p, out.Ac.v.p);
  AMG_LAUNCH_CHECK();
  AMG_HIP(hipStreamSynchronize(s));
  tm.rap_ms += now_ms() - t1;
}

void finish_level(Level &Lv, hipStream_t s, bool want_float, bool want_codes) {
  const int n = Lv.A.n;
  Lv.dinv.alloc(n);
  hipLaunchKernelGGL(k_l1_dinv, grid_for(n), dim3(kBlock), 0, s, n, Lv.A.rp.p, Lv.A.v.p, Lv.dinv.p);
  AMG_LAUNCH_CHECK();
  build_sell(Lv, s, want_float, want_codes);
  if (want_float) {
    Lv.dinvf.alloc(n);
    hipLaunchKernelGGL(k_l1_dinv_f, grid_for(n), dim3(kBlock), 0, s, n, Lv.A.rp.p, Lv.A.v.p, Lv.dinvf.p);
    AMG_LAUNCH_CHECK();
  }
}

void build_members(Level &Lv, hipStream_t s) {
  const int n = Lv.A.n, nc = Lv.nc;
  tvec<int> cnt(nc, s), fill(nc, s);
  AMG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * nc, s));
  AMG_HIP(hipMemsetAsync(fill.p, 0, sizeof(int) * nc, s));
  hipLaunchKernelGGL(k_count_members, grid_for(n), dim3(kBlock), 0, s, n, Lv.agg.p, cnt.p);
  AMG_LAUNCH_CHECK();
  Lv.mptr.alloc(nc + 1);
  exclusive_scan(cnt.p, Lv.mptr.p, nc, s);
  Lv.mem.alloc(n);
  hipLaunchKernelGGL(k_place_members, grid_for(n), dim3(kBlock), 0, s, n, Lv.agg.p, Lv.mptr.p, fill.p,
                     Lv.mem.p);
  hipLaunchKernelGGL(k_sort_members, grid_for(nc), dim3(kBlock), 0, s, nc, Lv.mptr.p, Lv.mem.p);
  AMG_LAUNCH_CHECK();
}

}  // namespace

// Pool memory freed by setup temporaries stays cached up to this amount, so
// repeated setups do not map and unmap memory.
constexpr uint64_t kPoolKeepBytes = 8ull << 30;

void keep_pool_memory() {
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::vector<int> done;
  std::lock_guard<std::mutex> lock(mu);
  if (static_cast<int>(done.size()) <= dev) done.resize(dev + 1, 0);
  if (done[dev]) return;
  hipMemPool_t pool;
  AMG_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = kPoolKeepBytes;
  AMG_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  done[dev] = 1;
}

// Entry points for the other translation units (batched hierarchy).
void device_exclusive_scan(const int *in, int *out, int n, hipStream_t s) { exclusive_scan(in, out, n, s); }
int device_read_int(const int *p, hipStream_t s) { return read_int(p, s); }
void finalize_level(Level &Lv, hipStream_t s, bool want_float, bool want_codes) {
  finish_level(Lv, s, want_float, want_codes);
}
double wall_ms() { return now_ms(); }

// ================================================= bootstrap composite
// Appendix A's bootstrap AMG: while the composite of the hierarchies built so
// far has fewer than max_hrc members and its estimated convergence rate is
// above bootstrap_rate, the iterate that estimate ends with (the error the
// composite reduces slowest), scaled by its largest magnitude, becomes the
// smooth vector of one more hierarchy with the same parameters.  Estimate:
// bootstrap_its steps x <- x + B (0 - A x) on A x = 0 from a SplitMix64 start
// vector, rate = (||x_its||_A / ||x_0||_A)^(1 / its).

// SplitMix64 (Steele, Lea and Flood 2014): first output for state c.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long c) {
  unsigned long long z = c + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// x_i = 2 u - 1, u = (splitmix64(((16 seed + j) << 32) + i) >> 11) 2^-53
__global__ void k_bootstrap_start(int n, unsigned seed16j, double *x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long c = (static_cast<unsigned long long>(seed16j) << 32) + static_cast<unsigned>(i);
  const double u = static_cast<double>(splitmix64(c) >> 11) * 0x1.0p-53;
  x[i] = 2.0 * u - 1.0;
}

__global__ void k_neg_from_zero(int n, double *t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = 0.0 - t[i];
}

__global__ void k_accumulate(int n, double *x, const double *e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = x[i] + e[i];
}

constexpr int kDotBlocks = 1024;

// Partial sums of x . y, one per workgroup (grid-stride), folded by k_dot_finish.
__global__ void __launch_bounds__(kBlock) k_dot_part(int n, const double *x, const double *y, double *part) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) acc = acc + x[i] * y[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kBlock) k_dot_finish(int np, const double *part, double *out) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int q = threadIdx.x; q < np; q += kBlock) acc = acc + part[q];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

namespace {
double device_dot(int n, const double *x, const double *y, double *part, double *res, hipStream_t s) {
  const int nb = std::max(1, std::min(kDotBlocks, ceil_div(n, kBlock)));
  hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(kBlock), 0, s, n, x, y, part);
  hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(kBlock), 0, s, nb, part, res);
  AMG_LAUNCH_CHECK();
  double v = 0.0;
  read_small(&v, res, sizeof(double), s);
  return v;
}
}  // namespace

void destroy_components(amg_hierarchy *h) {
  for (amg_hierarchy *c : h->comp) {
    destroy_graph(c);
    if (c->sc_host) (void)hipHostFree(c->sc_host);
    c->sc_host = nullptr;
    delete c;
  }
  h->comp.clear();
}

void bootstrap_build(amg_hierarchy *h) {
  const amg_params &P = h->p;
  if (P.max_hrc <= 1 || !P.precond) return;
  hipStream_t s = h->stream;
  const double t0 = now_ms();
  const int n = h->L[0].A.n;
  h->ct.alloc(n);
  h->ce.alloc(n);
  dvec<double> x(n), t(n), e(n), part(kDotBlocks), res(1);
  dvec<unsigned long long> mx(1);
  dvec<int> nf(1);
  // the components are built from the fine matrix the head already holds
  const DevCSR &A0 = h->L[0].A;
  amg_csr Adev{n, A0.nnz, A0.rp.p, A0.ci.p, A0.v.p, 1};
  const dim3 g = grid_for(n), b(kBlock);
  auto a_norm = [&](const double *v) {
    enqueue_spmv(h, 0, v, t.p);
    return sqrt(device_dot(n, v, t.p, part.p, res.p, s));
  };
  for (;;) {
    const int m = 1 + static_cast<int>(h->comp.size());
    hipLaunchKernelGGL(k_bootstrap_start, g, b, 0, s, n, static_cast<unsigned>(16 * P.bootstrap_seed + m), x.p);
    AMG_LAUNCH_CHECK();
    const double n0 = a_norm(x.p);
    for (int it = 0; it < P.bootstrap_its; ++it) {
      enqueue_spmv(h, 0, x.p, t.p);
      hipLaunchKernelGGL(k_neg_from_zero, g, b, 0, s, n, t.p);
      enqueue_composite(h, m, t.p, e.p);
      hipLaunchKernelGGL(k_accumulate, g, b, 0, s, n, x.p, e.p);
      AMG_LAUNCH_CHECK();
    }
    const double nfin = a_norm(x.p);
    const double rate = pow(nfin / n0, 1.0 / static_cast<double>(P.bootstrap_its));
    h->rates.push_back(rate);
    if (rate <= P.bootstrap_rate || m >= P.max_hrc) break;
    AMG_HIP(hipMemsetAsync(mx.p, 0, sizeof(unsigned long long), s));
    AMG_HIP(hipMemsetAsync(nf.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_absmax, dim3(std::min(1024, ceil_div(n, kBlock))), b, 0, s, n, x.p, mx.p, nf.p);
    AMG_LAUNCH_CHECK();
    unsigned long long mbits = 0;
    read_small(&mbits, mx.p, sizeof(mbits), s);
    if (read_int(nf.p, s) || mbits == 0) break;   // non-finite or zero: no new vector
    hipLaunchKernelGGL(k_scale_by_max, g, b, 0, s, n, x.p, mx.p);
    AMG_LAUNCH_CHECK();
    amg_hierarchy *c = new amg_hierarchy();
    h->comp.push_back(c);
    c->p = P;
    c->p.smooth_vec = AMG_SMOOTH_GIVEN;
    c->p.smooth_vector = x.p;
    c->p.max_hrc = 1;
    c->stream = s;
    c->dev = h->dev;
    build_hierarchy(c, &Adev);
    c->p.smooth_vector = nullptr;
  }
  AMG_HIP(hipStreamSynchronize(s));
  h->tm.bootstrap_ms = now_ms() - t0;
  h->tm.setup_ms += h->tm.bootstrap_ms;
}

// ===================================================== hierarchy builder
void build_hierarchy(amg_hierarchy *h, const amg_csr *Ain) {
  hipStream_t s = h->stream;
  const amg_params &P = h->p;
  const double t_start = now_ms();
  const bool want_float = (P.precision == AMG_PREC_MIXED);
  h->L.clear();
  h->L.emplace_back();
  Level &L0 = h->L[0];
  const int n = Ain->n;
  L0.A.n = n;
  L0.A.nnz = Ain->nnz;
  L0.A.rp.alloc(n + 1);
  L0.A.ci.alloc(Ain->nnz);
  L0.A.v.alloc(Ain->nnz);
  const hipMemcpyKind kind = Ain->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  AMG_HIP(hipMemcpyAsync(L0.A.rp.p, Ain->row_ptr, sizeof(int) * (n + 1), kind, s));
  AMG_HIP(hipMemcpyAsync(L0.A.ci.p, Ain->col_idx, sizeof(int) * Ain->nnz, kind, s));
  AMG_HIP(hipMemcpyAsync(L0.A.v.p, Ain->val, sizeof(double) * Ain->nnz, kind, s));
  {
    dvec<int> flags(4);
    AMG_HIP(hipMemsetAsync(flags.p, 0, sizeof(int) * 4, s));
    hipLaunchKernelGGL(k_validate_rows, grid_for(n), dim3(kBlock), 0, s, n, Ain->nnz, L0.A.rp.p,
                       L0.A.ci.p, L0.A.v.p, flags.p);
    AMG_LAUNCH_CHECK();
    check_flags(flags, s);
    hipLaunchKernelGGL(k_validate_sym, grid_for(n), dim3(kBlock), 0, s, n, L0.A.rp.p, L0.A.ci.p,
                       L0.A.v.p, flags.p);
    AMG_LAUNCH_CHECK();
    check_flags(flags, s);
  }
  const bool want_codes = P.value_coding == AMG_VALUES_AUTO;
  finish_level(L0, s, want_float, want_codes);

  // smooth vector of the fine level
  AMG_HIP(hipStreamSynchronize(s));
  const double t_w = now_ms();
  L0.w.alloc(n);
  // The learned vector (the network's prediction from the fine matrix) is
  // used when every entry is finite and positive; otherwise the setup falls
  // back to relaxation and records AMG_ERR_MODEL in amg_info.smooth_status.
  bool relax = (P.smooth_vec == AMG_SMOOTH_RELAX);
  h->smooth_status = AMG_OK;
  if (P.smooth_vec == AMG_SMOOTH_LEARNED) {
    const amg_csr Adev{n, L0.A.nnz, L0.A.rp.p, L0.A.ci.p, L0.A.v.p, 1};
    std::vector<float> from_file;
    const float *theta = P.model_params;
    int st = AMG_OK;
    if (!theta) {   // the parameters from model_path
      from_file.resize(AMG_MPNN_NPARAMS);
      st = mpnn_read_params_file(P.model_path, from_file.data()) ? AMG_OK : AMG_ERR_MODEL;
      theta = from_file.data();
    }
    if (st == AMG_OK) st = mpnn_predict_for_setup(theta, &Adev, L0.w.p, s);
    if (st == AMG_OK) {
      dvec<int> flag(1);
      AMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
      hipLaunchKernelGGL(k_check_usable, grid_for(n), dim3(kBlock), 0, s, n, L0.w.p, flag.p);
      AMG_LAUNCH_CHECK();
      if (read_int(flag.p, s)) st = AMG_ERR_MODEL;
    } else if (st == AMG_ERR_NOMEM || st == AMG_ERR_DEVICE) {
      fail(st, "learned smooth vector: " + api_last_error());
    }
    if (st != AMG_OK) {
      h->smooth_status = AMG_ERR_MODEL;
      relax = true;
    }
  }
  if (P.smooth_vec == AMG_SMOOTH_GIVEN) {
    AMG_HIP(hipMemcpyAsync(L0.w.p, P.smooth_vector, sizeof(double) * n, kind, s));
    dvec<int> flag(1);
    AMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_check_finite, grid_for(n), dim3(kBlock), 0, s, n, L0.w.p, flag.p);
    AMG_LAUNCH_CHECK();
    if (read_int(flag.p, s)) fail(AMG_ERR_NONFINITE, "non-finite smooth vector");
  } else if (P.smooth_vec != AMG_SMOOTH_LEARNED || relax) {
    hipLaunchKernelGGL(k_fill, grid_for(n), dim3(kBlock), 0, s, n, L0.w.p, 1.0);
    AMG_LAUNCH_CHECK();
    if (relax) {
      dvec<double> t(n), zero(n);
      AMG_HIP(hipMemsetAsync(zero.p, 0, sizeof(double) * n, s));
      for (int it = 0; it < P.smooth_sweeps; ++it) {
        enqueue_sweep(h, 0, zero.p, L0.w.p, t.p);   // w <- w + dinv (0 - A w)
        std::swap(L0.w, t);
      }
      dvec<unsigned long long> mx(1);
      dvec<int> nf(1);
      AMG_HIP(hipMemsetAsync(mx.p, 0, sizeof(unsigned long long), s));
      AMG_HIP(hipMemsetAsync(nf.p, 0, sizeof(int), s));
      hipLaunchKernelGGL(k_absmax, dim3(std::min(1024, ceil_div(n, kBlock))), dim3(kBlock), 0, s, n, L0.w.p,
                         mx.p, nf.p);
      AMG_LAUNCH_CHECK();
      if (read_int(nf.p, s)) {
        hipLaunchKernelGGL(k_fill, grid_for(n), dim3(kBlock), 0, s, n, L0.w.p, 1.0);
      } else {
        hipLaunchKernelGGL(k_scale_by_max, grid_for(n), dim3(kBlock), 0, s, n, L0.w.p, mx.p);
      }
      AMG_LAUNCH_CHECK();
    }
  }
  AMG_HIP(hipStreamSynchronize(s));
  h->tm.smooth_ms = now_ms() - t_w;

  Arena ws;   // setup temporaries of the pairwise steps (largest first)
  // decoupled aggregation: row-block bounds of the current level (Sec. 4.1)
  const int nparts = P.n_parts;
  dvec<int> off_level;
  if (nparts > 1) {
    std::vector<int> off(nparts + 1);
    for (int q = 0; q <= nparts; ++q) off[q] = static_cast<int>(static_cast<int64_t>(q) * n / nparts);
    off_level.alloc(nparts + 1);
    AMG_HIP(hipMemcpyAsync(off_level.p, off.data(), sizeof(int) * (nparts + 1), hipMemcpyHostToDevice, s));
    AMG_HIP(hipStreamSynchronize(s));
  }
  const int maxlev = std::min(P.max_levels, AMG_MAX_LEVELS);
  while (P.precond && static_cast<int>(h->L.size()) < maxlev && h->L.back().A.n > P.coarse_max) {
    const int k = static_cast<int>(h->L.size()) - 1;
    const int nk = h->L[k].A.n;
    dvec<int> agg(nk);
    dvec<double> pv(nk);
    hipLaunchKernelGGL(k_iota, grid_for(nk), dim3(kBlock), 0, s, nk, agg.p, pv.p);
    AMG_LAUNCH_CHECK();
    PairStep cur;          // owns the intermediate matrix after step 0
    bool owned = false;
    for (int step = 0; step < P.aggr_steps; ++step) {
      const DevCSR &Acur = owned ? cur.Ac : h->L[k].A;
      const double *wcur = owned ? cur.wc.p : h->L[k].w.p;
      const int *offcur = nparts > 1 ? (owned ? cur.offc.p : off_level.p) : nullptr;
      if (step > 0 && Acur.n <= P.coarse_max) break;
      PairStep nxt;
      pairwise_step(Acur, wcur, offcur, nparts, s, nxt, h->tm, ws);
      hipLaunchKernelGGL(k_compose, grid_for(nk), dim3(kBlock), 0, s, nk, agg.p, pv.p, nxt.agg.p,
                         nxt.p.p);
      AMG_LAUNCH_CHECK();
      AMG_HIP(hipStreamSynchronize(s));
      cur = std::move(nxt);
      owned = true;
    }
    if (!owned || static_cast<double>(cur.Ac.n) > kStagnation * static_cast<double>(nk)) break;
    Level &Lk = h->L[k];
    Lk.nc = cur.Ac.n;
    Lk.agg = std::move(agg);
    Lk.pval = std::move(pv);
    build_members(Lk, s);
    if (want_float) {
      Lk.pvalf.alloc(nk);
      hipLaunchKernelGGL(k_d2f, grid_for(nk), dim3(kBlock), 0, s, static_cast<int64_t>(nk),
                         Lk.pval.p, Lk.pvalf.p);
      AMG_LAUNCH_CHECK();
    }
    if (want_codes) build_pcodes(Lk, s);
    if (nparts > 1) off_level = std::move(cur.offc);
    Level next;
    next.A = std::move(cur.Ac);
    next.w = std::move(cur.wc);
    h->L.push_back(std::move(next));
    finish_level(h->L.back(), s, want_float, want_codes);
  }
  AMG_HIP(hipStreamSynchronize(s));
  coarse_factor(h);
  alloc_solve_buffers(h);
  AMG_HIP(hipStreamSynchronize(s));
  h->tm.setup_ms = now_ms() - t_start;
}

void coarse_factor(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  Level &C = h->L.back();
  const int n = C.A.n;
  h->coarse_dense = h->p.precond && h->p.coarse_solver == AMG_COARSE_CHOLESKY && n <= kDenseMax;
  if (!h->coarse_dense) return;
  const int64_t nn = static_cast<int64_t>(n) * n;
  dvec<double> D(nn);
  dvec<int> flag(1);
  AMG_HIP(hipMemsetAsync(D.p, 0, sizeof(double) * nn, s));
  AMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_densify, grid_for(n), dim3(kBlock), 0, s, n, C.A.rp.p, C.A.ci.p, C.A.v.p, D.p);
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, s, n, D.p, flag.p);
  AMG_LAUNCH_CHECK();
  if (read_int(flag.p, s)) fail(AMG_ERR_NOT_SPD, "coarsest matrix has a non-positive Cholesky pivot");
  h->Ainv.alloc(nn);
  dvec<double> Dt(nn);
  hipLaunchKernelGGL(k_transpose_sq, grid_for(nn), dim3(kBlock), 0, s, n, D.p, Dt.p);
  hipLaunchKernelGGL(k_chol_inverse, dim3(ceil_div(n, kInvCols)), dim3(kWave), 0, s, n, D.p, Dt.p,
                     h->Ainv.p);
  AMG_LAUNCH_CHECK();
  AMG_HIP(hipStreamSynchronize(s));
}

}  // namespace amg
