// Internal definitions shared by the HIP translation units of libamg355.
// Not part of the public ABI (include/amg355.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "amg355.h"

namespace amg {

// ------------------------------------------------------------------ errors

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);

#define AMG_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      ::amg::fail(e_ == hipErrorOutOfMemory ? AMG_ERR_NOMEM : AMG_ERR_DEVICE,             \
                  std::string(#call) + ": " + hipGetErrorString(e_));                     \
  } while (0)

#define AMG_LAUNCH_CHECK() AMG_HIP(hipGetLastError())

// --------------------------------------------------------- device buffers

// Owning device array.  Moves only.
template <class T>
struct dvec {
  T *p = nullptr;
  size_t n = 0;
  hipStream_t st = nullptr;   // stream of a pooled allocation
  bool pooled = false;
  dvec() = default;
  explicit dvec(size_t count) { alloc(count); }
  dvec(const dvec &) = delete;
  dvec &operator=(const dvec &) = delete;
  dvec(dvec &&o) noexcept : p(o.p), n(o.n), st(o.st), pooled(o.pooled) { o.p = nullptr; o.n = 0; }
  dvec &operator=(dvec &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; st = o.st; pooled = o.pooled;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~dvec() { release(); }
  void alloc(size_t count);
  void release();
  size_t bytes() const { return sizeof(T) * n; }
  T *get() const { return p; }
};

// While a PoolScope is alive on a host thread, the dvec allocations it makes
// come from the device's memory pool, ordered on the scope's stream, and are
// freed in order on that stream (which must outlive them): no device-wide
// synchronisation per allocation or free, and memory released by one
// hierarchy is reused by the next.  Outside a scope dvec uses hipMalloc.
struct PoolScope {
  static hipStream_t &stream() {
    static thread_local hipStream_t s = nullptr;
    return s;
  }
  static bool &active() {
    static thread_local bool on = false;
    return on;
  }
  // stream on which pooled releases are ordered instead of their own (set
  // by FreeOn), or null
  static hipStream_t &free_override() {
    static thread_local hipStream_t s = nullptr;
    return s;
  }
  hipStream_t prev_s;
  bool prev_on;
  explicit PoolScope(hipStream_t s) : prev_s(stream()), prev_on(active()) {
    stream() = s;
    active() = true;
  }
  ~PoolScope() {
    stream() = prev_s;
    active() = prev_on;
  }
  PoolScope(const PoolScope &) = delete;
  PoolScope &operator=(const PoolScope &) = delete;
};

// Allocations made while a NoPool is alive use hipMalloc even inside a
// PoolScope: for buffers that outlive the scope's stream (per-thread caches).
struct NoPool {
  bool prev;
  NoPool() : prev(PoolScope::active()) { PoolScope::active() = false; }
  ~NoPool() { PoolScope::active() = prev; }
  NoPool(const NoPool &) = delete;
  NoPool &operator=(const NoPool &) = delete;
};

// Pooled releases made while a FreeOn is alive are ordered on its stream,
// for objects whose own stream is synchronised and may not outlive them.
struct FreeOn {
  hipStream_t prev;
  explicit FreeOn(hipStream_t s) : prev(PoolScope::free_override()) { PoolScope::free_override() = s; }
  ~FreeOn() { PoolScope::free_override() = prev; }
  FreeOn(const FreeOn &) = delete;
  FreeOn &operator=(const FreeOn &) = delete;
};

// The library's own streams on the current device (slot 0: the stream of
// hierarchies given none; slots 1..kBuildThreads: setup worker threads):
// created on first use and kept for the life of the process (pool memory
// freed on a stream must not outlive it).  Blocking streams, so they stay
// ordered with null-stream work.  nullptr if one cannot be created.
constexpr int kBuildThreads = 8;   // host threads building a batch's hierarchies
hipStream_t library_stream(int slot = 0);

// The stream of a hierarchy or batch created without a caller stream: one
// per live object, so that objects used from different host threads at once
// do not serialise on one stream (each solve synchronises its object's
// stream).  Also the setup stream that stands in for a caller's stream
// (SetupStream) and the capture streams (capture_graph).  Kept
// for the life of the process and handed out again once their object is
// destroyed.  acquire: nullptr if none can be created; *dev receives the
// current device, which release needs back.
hipStream_t acquire_private_stream(int *dev, unsigned flags = hipStreamDefault);
void release_private_stream(int dev, hipStream_t s, unsigned flags = hipStreamDefault);

// Records into *graph the work enqueue() puts on `stream` (an object's
// stream field), through a non-blocking stream swapped in for the capture.
// A blocking stream that is capturing would make the null stream depend on
// the capture, and the runtime then refuses work on every other blocking
// stream, other host threads' included; a non-blocking stream stays outside
// that synchronisation.  Nothing executes on the capture stream (taken from
// and returned to the library's free list); the graph is launched on
// `stream` afterwards.
template <class F>
void capture_graph(hipStream_t &stream, hipGraph_t *graph, F enqueue) {
  struct Swap {
    hipStream_t &slot, orig, cs = nullptr;
    int dev = 0;
    bool capturing = false;
    ~Swap() {
      if (capturing) {   // enqueue threw: end the capture and drop what it recorded
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(cs, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      }
      slot = orig;
      release_private_stream(dev, cs, hipStreamNonBlocking);
    }
  } sw{stream, stream};
  sw.cs = acquire_private_stream(&sw.dev, hipStreamNonBlocking);
  if (!sw.cs) fail(AMG_ERR_DEVICE, "hipStreamCreateWithFlags failed");
  AMG_HIP(hipStreamBeginCapture(sw.cs, hipStreamCaptureModeThreadLocal));
  sw.capturing = true;
  stream = sw.cs;
  enqueue();
  sw.capturing = false;
  AMG_HIP(hipStreamEndCapture(sw.cs, graph));
}

// Runs an object's setup on a library stream that lives for the process in
// place of a caller's stream: every pooled block the setup frees (its
// temporaries) and every block the object keeps (freed at destroy) is then
// ordered on a stream that outlives it, whatever the caller later does with
// its own stream.  The setup stream first waits for the caller's stream (the
// input may be produced there); the destructor synchronises it, so the
// caller's stream sees a finished setup, and puts the caller's stream back.
// No-op when the object owns its stream already.
struct SetupStream {
  hipStream_t &slot;
  hipStream_t caller = nullptr, ss = nullptr;
  int dev = 0;
  SetupStream(hipStream_t &stream, bool callers_stream) : slot(stream) {
    if (!callers_stream) return;
    caller = stream;
    ss = acquire_private_stream(&dev);
    if (!ss) fail(AMG_ERR_DEVICE, "hipStreamCreate failed");
    hipEvent_t e = nullptr;
    hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventRecord(e, caller);
    if (err == hipSuccess) err = hipStreamWaitEvent(ss, e, 0);
    if (e) (void)hipEventDestroy(e);
    if (err != hipSuccess) {
      release_private_stream(dev, ss);
      fail(AMG_ERR_DEVICE, std::string("joining the caller's stream: ") + hipGetErrorString(err));
    }
    slot = ss;
  }
  ~SetupStream() {
    if (!ss) return;
    (void)hipStreamSynchronize(ss);
    slot = caller;
    release_private_stream(dev, ss);
  }
  SetupStream(const SetupStream &) = delete;
  SetupStream &operator=(const SetupStream &) = delete;
};

template <class T>
void dvec<T>::release() {
  if (p) {
    if (pooled) (void)hipFreeAsync(p, PoolScope::free_override() ? PoolScope::free_override() : st);
    else (void)hipFree(p);
  }
  p = nullptr;
  n = 0;
}

template <class T>
void dvec<T>::alloc(size_t count) {
  release();
  n = count;
  pooled = PoolScope::active();
  st = pooled ? PoolScope::stream() : nullptr;
  if (!count) return;
  if (pooled) AMG_HIP(hipMallocAsync(reinterpret_cast<void **>(&p), sizeof(T) * count, st));
  else AMG_HIP(hipMalloc(reinterpret_cast<void **>(&p), sizeof(T) * count));
}

// Stream-ordered scratch array for work inside one host function: allocated
// and freed in order on `s` from the device's memory pool (which keeps the
// memory for reuse), so temporaries cost no device-wide synchronisation.
template <class T>
struct tvec {
  T *p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  tvec() = default;
  tvec(size_t count, hipStream_t st) { alloc(count, st); }
  tvec(const tvec &) = delete;
  tvec &operator=(const tvec &) = delete;
  tvec(tvec &&o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
  tvec &operator=(tvec &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~tvec() { release(); }
  void alloc(size_t count, hipStream_t st) {
    release();
    n = count;
    s = st;
    if (count) AMG_HIP(hipMallocAsync(reinterpret_cast<void **>(&p), sizeof(T) * count, st));
  }
  void release() {
    if (p) (void)hipFreeAsync(p, s);
    p = nullptr;
    n = 0;
  }
};

// Keep freed pool memory cached for later setups (called once per device).
void keep_pool_memory();

// Grow-only device workspace carved into temporaries (256-byte aligned);
// reset() makes the whole buffer available again.  Work that used earlier
// carvings must be ordered before later users on the same stream.
struct Arena {
  dvec<unsigned char> buf;
  size_t off = 0;
  void reserve(size_t bytes) {
    if (buf.n < bytes) buf.alloc(bytes);
    off = 0;
  }
  void reset() { off = 0; }
  template <class T>
  T *take(size_t count) {
    const size_t a = (off + 255) & ~static_cast<size_t>(255);
    if (a + sizeof(T) * count > buf.n) fail(AMG_ERR_DEVICE, "setup workspace exhausted");
    off = a + sizeof(T) * count;
    return reinterpret_cast<T *>(buf.p + a);
  }
};

// A typed carving of an Arena (member `p` like the owning arrays).
template <class T>
struct wsv {
  T *p = nullptr;
  wsv() = default;
  wsv(Arena &a, size_t count) : p(a.take<T>(count)) {}
};

// ---------------------------------------------------------------- layouts

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kSlice = 64;         // SELL slice height = one wavefront of rows
constexpr int kBlock = 256;        // rows per workgroup in row-parallel kernels
constexpr int kXcd = 8;            // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kMaxDevices = 64;    // devices a process may use the library on
constexpr int kDenseMax = 1024;    // largest coarsest level factored densely
constexpr double kStagnation = 0.95;
constexpr int kTailRows = 1024;    // levels up to this size run in the coarse-tail kernel
constexpr int kTailThreads = 1024; // one row (and one aggregate) per thread
constexpr int kTailLds = 8192;     // LDS elements for the tail's vectors: 4 per row and level
static_assert(kTailRows <= kTailThreads, "the coarse tail maps one row to one thread");

// Canonical CSR (setup, export, next-level construction).
struct DevCSR {
  int n = 0;
  int64_t nnz = 0;
  dvec<int> rp, ci;
  dvec<double> v;
};

// Sliced ELLPACK with slice height 64 (one wavefront): row r of slice s keeps
// its k-th stored entry at slot sptr[s] + k*64 + (r % 64); slots past the end
// of a row hold col = r, val = 0.  Entry order within a row = CSR order.
struct Sell {
  int n = 0;
  int nslices = 0;
  int64_t nslots = 0;
  int wmin = 0, wmax = 0;   // narrowest and widest slice (slots per lane)
  dvec<int> sptr;     // nslices + 1 slot offsets (multiples of 64)
  dvec<int> col;
  dvec<double> val;
  dvec<float> valf;   // binary32 copy for the mixed-precision V-cycle
  // Compact column form read by the streaming kernels: the 64 slots k of a
  // slice (one "group", index sptr[s]/64 + k) share cbase[group] = smallest
  // column among them and keep col - cbase as 16 bits.  A slice whose group
  // spans more than 65535 columns keeps cbase = -1 on all its groups and is
  // read from `col`.  The 16-bit offsets (and the value codes below) are
  // stored by quads: slots 4t .. 4t+3 of one lane are adjacent, so a lane
  // reads four slots with one load.  Slot k of lane l in slice s sits at
  // ((qptr[s] + k/4) * 64 + l) * 4 + k%4; a slice holds ceil(width/4) quads
  // (padding slots 0).
  dvec<int> cbase;               // nslots / 64 + kGroupPad (the padding reads as 0)
  dvec<int> qptr;                // nslices + 1 quad offsets
  dvec<unsigned short> cdel;     // 256 per quad
  int64_t nquads = 0;
  int64_t nnz_compact = 0;       // matrix entries in compact slices
  int64_t groups_compact = 0;    // groups of compact slices
  // Coded values: when the slots (padding included) hold at most kDictMax
  // distinct bit patterns, each slot's byte indexes the level's table of
  // them, in ascending bit-pattern order (dict; dictf = its binary32 image),
  // and the streaming kernels read codes instead of val / valf.  Codes are
  // stored by quads like the 16-bit column offsets.  ndict = 0: plain.
  dvec<unsigned char> code;      // 256 per quad
  dvec<double> dict;
  dvec<float> dictf;
  int ndict = 0;
};

constexpr int kDictMax = 256;
constexpr int kGroupPad = 8;   // cbase entries past the last group, so 8-slot reads stay in range

// Value access of a SELL matrix as the kernels see it: val, or code + dict.
template <class T>
struct ValRef {
  const T *val;
  const unsigned char *code;   // null: read val
  const T *dict;
  int ndict;
};

// Column access of a SELL matrix as the kernels see it.
struct SellRef {
  const int *sptr, *col, *cbase, *qptr;
  const unsigned short *cdel;   // null: all slices read `col`
};
inline SellRef sell_ref(const Sell &S) { return SellRef{S.sptr.p, S.col.p, S.cbase.p, S.qptr.p, S.cdel.p}; }
template <class T>
ValRef<T> val_ref(const Sell &S);
template <>
inline ValRef<double> val_ref<double>(const Sell &S) {
  return ValRef<double>{S.val.p, S.ndict ? S.code.p : nullptr, S.dict.p, S.ndict};
}
template <>
inline ValRef<float> val_ref<float>(const Sell &S) {
  return ValRef<float>{S.valf.p, S.ndict ? S.code.p : nullptr, S.dictf.p, S.ndict};
}

struct Level {
  DevCSR A;
  Sell S;
  dvec<double> dinv, w;
  dvec<float> dinvf;
  // transfer to level k+1 (empty on the coarsest level)
  int nc = 0;
  dvec<int> agg;          // n: coarse row of fine row i
  dvec<double> pval;      // n: value of P(i, agg[i])
  dvec<float> pvalf;
  // P values as codes (coded hierarchies, at most kDictMax distinct values):
  // pval[i] = pdict[pcode[i]] bit for bit; npdict = 0: read pval
  dvec<unsigned char> pcode;
  dvec<double> pdict;
  int npdict = 0;
  dvec<int> mptr, mem;    // CSR of P^T: members of each aggregate, ascending
  // V-cycle work vectors
  dvec<double> r, x, t;
  dvec<float> rf, xf, tf;
  // general cycle (H/W cycles, Jacobi / Gauss-Seidel smoothers): 1 / a_ii,
  // the second coarse correction's vectors, the Gauss-Seidel level schedule
  dvec<double> djac, ge, gw, gz;
  dvec<int> gs_rows, gs_ptr_d;
  std::vector<int> gs_ptr;
};

struct Scalars {        // PCG state living in device memory
  double rho, c, a, rr, nr0, thr, alpha, beta, gamma;
  int it;       // preconditioner applications so far
  int done;     // 1 once converged, broken down or at maxit
  int status;   // 0 or an AMG_ERR_* code
  int conv;     // 1 if ||r|| <= rtol ||r_0|| was reached
  int maxit;
  int pad;
};

// P values as a kernel reads them: pval[i], or pdict[pcode[i]] when coded.
template <class T>
struct PVals {
  const T *pval;
  const unsigned char *pcode;   // null: read pval
  const T *pdict;
#ifdef __HIPCC__
  __device__ __forceinline__ T operator()(int i) const { return pcode ? pdict[pcode[i]] : pval[i]; }
#endif
};

// Device-side description of one level for the coarse-tail kernel.
template <class T>
struct TailDesc {
  int n, nc;
  int lds;          // offset (elements of T) of the level's four LDS vectors
  const int *sptr, *col;
  const T *val, *pval;
  const int *agg, *mptr, *mem;
};

struct Timing {
  double setup_ms = 0, match_ms = 0, rap_ms = 0, smooth_ms = 0, bootstrap_ms = 0;
  int rounds = 0;
};

}  // namespace amg

struct amg_hierarchy {
  amg_params p{};
  hipStream_t stream = nullptr;
  bool own_stream = false;     // stream from acquire_private_stream (on stream_dev)
  int stream_dev = 0;
  int dev = 0;                 // device current at amg_setup (holds every buffer)
  std::vector<amg::Level> L;
  int coarse_dense = 0;
  amg::dvec<double> Ainv;      // inverse of the coarsest matrix, column-major
  // levels [tail_start, levels) run inside one workgroup (coarse-tail kernel)
  int tail_start = 0;
  int tail_w = 0;              // widest SELL slice (slots) among the tail levels
  bool tail_general = false;   // the tail runs the general cycle (k_cycle_tail_g, 5 vectors per level)
  amg::dvec<unsigned char> tail_desc_d, tail_desc_f;   // TailDesc<double> / <float> arrays
  // PCG vectors
  amg::dvec<double> u, r, w, v, d, q;
  amg::dvec<double> partials;  // 3 per workgroup of the fine-level reductions
  amg::dvec<amg::Scalars> sc;
  amg::Scalars *sc_host = nullptr;   // pinned, host-coherent mirror written by the GPU
  amg::Scalars *sc_host_dev = nullptr;   // device address of sc_host
  amg::Timing tm;
  // hipGraph of one PCG iteration (V-cycle + SpMV/dots + update)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int use_graph = 1;
  // bootstrap composite: hierarchies 2..m (owned; they run on this
  // hierarchy's stream), the rate estimates, and two fine-level work vectors
  int smooth_status = AMG_OK;  // AMG_ERR_MODEL: the learned vector was unusable
  std::vector<amg_hierarchy *> comp;
  std::vector<double> rates;
  amg::dvec<double> ct, ce;
};

namespace amg {

// ------------------------------------------------------- setup interface
void build_hierarchy(amg_hierarchy *h, const amg_csr *A);
void coarse_factor(amg_hierarchy *h);
void device_exclusive_scan(const int *in, int *out, int n, hipStream_t s);  // out: n+1 entries
int device_read_int(const int *p, hipStream_t s);
void finalize_level(Level &Lv, hipStream_t s, bool want_float, bool want_codes);  // l1 diagonal + SELL from Lv.A
double wall_ms();

// -------------------------------------------------------- solve interface
void alloc_solve_buffers(amg_hierarchy *h);
void enqueue_vcycle(amg_hierarchy *h, const double *r, double *z);          // the preconditioner
void enqueue_vcycle_single(amg_hierarchy *h, const double *r, double *z);   // h's own V-cycle
// the first m hierarchies' composite with binary64 cycles (bootstrap estimates)
void enqueue_composite(amg_hierarchy *h, int m, const double *r, double *z);
// Network prediction inside amg_setup (per-device cached network; mpnn.hip).
int mpnn_predict_for_setup(const float *params, const amg_csr *A, double *w_out, hipStream_t s);
// AMG_MPNN_NPARAMS parameters from a model file into out; false when the file
// cannot be read or does not hold them (host only; mpnn.hip).
bool mpnn_read_params_file(const char *path, float *out);
void bootstrap_build(amg_hierarchy *h);   // adds hierarchies per max_hrc / bootstrap_rate
void destroy_components(amg_hierarchy *h);
void enqueue_spmv(amg_hierarchy *h, int k, const double *x, double *y);
void enqueue_sweep(amg_hierarchy *h, int k, const double *r, const double *x, double *xn);
int pcg_solve(amg_hierarchy *h, const double *b, double *x, double rtol, int maxit, int *iters,
              double *relres);
// amg_pcg_solve_noalloc: the same solve with its PCG state in a static
// per-device scratch array; noalloc_scratch(dev) looks up (once per device)
// and returns that array's device address.
int pcg_solve_noalloc(amg_hierarchy *h, const double *b, double *x, double rtol, int maxit,
                      int *iters, double *relres);
void *noalloc_scratch(int dev);
int64_t noalloc_max_rows();
void time_kernel(amg_hierarchy *h, int kernel, int k, int reps, double *avg_ms, double *bytes);
void destroy_graph(amg_hierarchy *h);

// --------------------------------------------------- C ABI error plumbing
int api_set_error(int code, const std::string &msg);
int api_check_params(const amg_params *p);        // AMG_OK or the status (message set)
int api_guarded(const std::function<int()> &f);   // maps amg::Error to a status
const std::string &api_last_error();

// ----------------------------------------------------------- small helpers
inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }
int64_t device_bytes(const amg_hierarchy *h);

}  // namespace amg

// ------------------------------------------------------ device-side helpers
#ifdef __HIPCC__
namespace amg {
// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b -> XCD
// b % 8).  Remap so that each XCD walks one contiguous range of logical
// blocks: neighbouring rows then share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  int per = nb / kXcd, rem = nb % kXcd;
  int x = b % kXcd, j = b / kXcd;
  return x * per + (x < rem ? x : rem) + j;
}

template <class T>
__device__ __forceinline__ T ld_stream(const T *p) {
  return __builtin_nontemporal_load(p);
}

// Deterministic sum over a 64-lane wavefront (fixed xor-butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
  return v;
}
}  // namespace amg
#endif
