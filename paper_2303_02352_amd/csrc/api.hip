// C ABI entry points (include/amg355.h).  Every function catches the
// library's internal errors and returns a status code; nothing is thrown
// across the boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "amg_internal.hpp"

namespace {
thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

template <class F>
int guarded(F &&f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const amg::Error &e) {
    return set_error(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    return set_error(AMG_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return set_error(AMG_ERR_DEVICE, "unexpected internal error");
  }
}

int check_params(const amg_params *p) {
  if (p->aggr_steps < 1 || p->max_levels < 1 || p->coarse_max < 1 || p->coarse_sweeps < 1 ||
      p->pre_sweeps < 0 || p->post_sweeps < 0 || p->smooth_sweeps < 0)
    return set_error(AMG_ERR_INVALID, "parameter out of range");
  if (p->coarse_solver != AMG_COARSE_CHOLESKY && p->coarse_solver != AMG_COARSE_JACOBI)
    return set_error(AMG_ERR_INVALID, "unknown coarse_solver");
  if (p->smooth_vec < AMG_SMOOTH_ONES || p->smooth_vec > AMG_SMOOTH_LEARNED)
    return set_error(AMG_ERR_INVALID, "unknown smooth_vec");
  if (p->smooth_vec == AMG_SMOOTH_GIVEN && !p->smooth_vector)
    return set_error(AMG_ERR_INVALID, "smooth_vec = GIVEN needs smooth_vector");
  if (p->smooth_vec == AMG_SMOOTH_LEARNED && !p->model_params && !p->model_path)
    return set_error(AMG_ERR_INVALID, "smooth_vec = LEARNED needs model_params or model_path");
  if (p->precision != AMG_PREC_DOUBLE && p->precision != AMG_PREC_MIXED)
    return set_error(AMG_ERR_INVALID, "unknown precision");
  if (p->value_coding != AMG_VALUES_PLAIN && p->value_coding != AMG_VALUES_AUTO)
    return set_error(AMG_ERR_INVALID, "unknown value_coding");
  if (p->precond != 0 && p->precond != 1) return set_error(AMG_ERR_INVALID, "precond must be 0 or 1");
  if (p->n_parts < 1 || p->n_parts > (1 << 24)) return set_error(AMG_ERR_INVALID, "n_parts out of range");
  if (p->cycle_type < AMG_CYCLE_V || p->cycle_type > AMG_CYCLE_W)
    return set_error(AMG_ERR_INVALID, "unknown cycle_type");
  auto relax_ok = [](int r) {
    return r == AMG_RELAX_JACOBI || r == AMG_RELAX_GS || r == AMG_RELAX_SYM_GS || r == AMG_RELAX_L1_JACOBI;
  };
  if (!relax_ok(p->relax_type) || !relax_ok(p->coarse_relax))
    return set_error(AMG_ERR_INVALID, "unknown relax_type or coarse_relax");
  if (p->max_hrc < 1 || p->max_hrc > 16) return set_error(AMG_ERR_INVALID, "max_hrc out of range");
  if (p->bootstrap_type < AMG_BOOTSTRAP_MULT || p->bootstrap_type > AMG_BOOTSTRAP_ADD)
    return set_error(AMG_ERR_INVALID, "unknown bootstrap_type");
  if (p->bootstrap_its < 1 || !(p->bootstrap_rate > 0.0 && p->bootstrap_rate <= 1.0))
    return set_error(AMG_ERR_INVALID, "bootstrap_its or bootstrap_rate out of range");
  if ((p->cycle_type != AMG_CYCLE_V || p->relax_type != AMG_RELAX_L1_JACOBI ||
       p->coarse_relax != AMG_RELAX_L1_JACOBI) && p->precision != AMG_PREC_DOUBLE)
    return set_error(AMG_ERR_UNSUPPORTED, "the binary32 cycle is the l1-Jacobi V-cycle");
  return AMG_OK;
}
}  // namespace

namespace amg {
void fail(int code, const std::string &msg) { throw Error{code, msg}; }
int api_check_params(const amg_params *p) { return check_params(p); }
int api_set_error(int code, const std::string &msg) { return set_error(code, msg); }
int api_guarded(const std::function<int()> &f) { return guarded(f); }
const std::string &api_last_error() { return g_last_error; }

int64_t device_bytes(const amg_hierarchy *h) {
  int64_t b = 0;
  for (const Level &L : h->L) {
    b += L.A.rp.bytes() + L.A.ci.bytes() + L.A.v.bytes();
    b += L.S.sptr.bytes() + L.S.col.bytes() + L.S.val.bytes() + L.S.valf.bytes();
    b += L.S.cbase.bytes() + L.S.cdel.bytes() + L.S.qptr.bytes();
    b += L.S.code.bytes() + L.S.dict.bytes() + L.S.dictf.bytes();
    b += L.dinv.bytes() + L.w.bytes() + L.dinvf.bytes() + L.agg.bytes() + L.pval.bytes();
    b += L.pvalf.bytes() + L.mptr.bytes() + L.mem.bytes();
    b += L.pcode.bytes() + L.pdict.bytes();
    b += L.r.bytes() + L.x.bytes() + L.t.bytes() + L.rf.bytes() + L.xf.bytes() + L.tf.bytes();
    b += L.djac.bytes() + L.ge.bytes() + L.gw.bytes() + L.gz.bytes() + L.gs_rows.bytes() + L.gs_ptr_d.bytes();
  }
  b += h->Ainv.bytes() + h->tail_desc_d.bytes() + h->tail_desc_f.bytes();
  b += h->u.bytes() + h->r.bytes() + h->w.bytes() + h->v.bytes() + h->d.bytes() + h->q.bytes();
  b += h->partials.bytes() + h->sc.bytes();
  return b;
}

hipStream_t library_stream(int slot) {
  int dev = 0;
  if (slot < 0 || slot > kBuildThreads || hipGetDevice(&dev) != hipSuccess) return nullptr;
  static std::mutex mu;
  static std::vector<hipStream_t> streams;   // (kBuildThreads + 1) per device
  std::lock_guard<std::mutex> lock(mu);
  const size_t at = static_cast<size_t>(dev) * (kBuildThreads + 1) + slot;
  if (streams.size() <= at) streams.resize(at + 1, nullptr);
  if (!streams[at] && hipStreamCreate(&streams[at]) != hipSuccess) streams[at] = nullptr;
  return streams[at];
}

namespace {
struct IdleStream {
  int dev;
  unsigned flags;
  hipStream_t s;
};
std::mutex g_private_mu;
std::vector<IdleStream> g_private_free;
}  // namespace

hipStream_t acquire_private_stream(int *dev, unsigned flags) {
  *dev = 0;
  if (hipGetDevice(dev) != hipSuccess) return nullptr;
  {
    std::lock_guard<std::mutex> lock(g_private_mu);
    for (size_t i = 0; i < g_private_free.size(); ++i)
      if (g_private_free[i].dev == *dev && g_private_free[i].flags == flags) {
        hipStream_t s = g_private_free[i].s;
        g_private_free.erase(g_private_free.begin() + static_cast<std::ptrdiff_t>(i));
        return s;
      }
  }
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, flags) != hipSuccess) return nullptr;
  return s;
}

void release_private_stream(int dev, hipStream_t s, unsigned flags) {
  if (!s) return;
  std::lock_guard<std::mutex> lock(g_private_mu);
  g_private_free.push_back(IdleStream{dev, flags, s});
}
}  // namespace amg

extern "C" {

int amg_params_default(amg_params *p) {
  if (!p) return set_error(AMG_ERR_INVALID, "NULL params");
  std::memset(p, 0, sizeof(*p));
  p->aggr_steps = 2;
  p->max_levels = 40;
  p->coarse_max = 100;
  p->coarse_solver = AMG_COARSE_CHOLESKY;
  p->coarse_sweeps = 20;
  p->pre_sweeps = 4;
  p->post_sweeps = 4;
  p->smooth_vec = AMG_SMOOTH_ONES;
  p->smooth_sweeps = 20;
  p->precond = 1;
  p->precision = AMG_PREC_DOUBLE;
  p->value_coding = AMG_VALUES_AUTO;
  p->n_parts = 1;
  p->cycle_type = AMG_CYCLE_V;
  p->relax_type = AMG_RELAX_L1_JACOBI;
  p->coarse_relax = AMG_RELAX_L1_JACOBI;
  p->max_hrc = 1;
  p->bootstrap_type = AMG_BOOTSTRAP_MULT;
  p->bootstrap_its = 15;
  p->bootstrap_seed = 1;
  p->bootstrap_rate = 0.8;
  p->smooth_vector = nullptr;
  p->model_params = nullptr;
  p->model_path = nullptr;
  p->stream = nullptr;
  return AMG_OK;
}

int amg_setup(const amg_csr *A, const amg_params *p, amg_hierarchy **h_out) {
  if (h_out) *h_out = nullptr;
  if (!A || !p || !h_out) return set_error(AMG_ERR_INVALID, "NULL argument");
  if (A->n <= 0 || A->nnz < A->n || A->nnz >= (int64_t(1) << 31) || !A->row_ptr || !A->col_idx ||
      !A->val)
    return set_error(AMG_ERR_INVALID, "bad CSR header (n, nnz or NULL array)");
  int st = check_params(p);
  if (st != AMG_OK) return st;
  amg_hierarchy *h = new (std::nothrow) amg_hierarchy();
  if (!h) return set_error(AMG_ERR_NOMEM, "host allocation failed");
  h->p = *p;
  if (p->stream) {
    h->stream = static_cast<hipStream_t>(p->stream);
  } else {
    // The null stream cannot be captured into a graph: work goes to a
    // blocking stream of the hierarchy's own, which stays ordered with
    // null-stream work.
    h->stream = amg::acquire_private_stream(&h->stream_dev);
    if (!h->stream) {
      delete h;
      return set_error(AMG_ERR_DEVICE, "no HIP device or stream available (hipGetDevice / hipStreamCreate failed)");
    }
    h->own_stream = true;
  }
  st = guarded([&] {
    AMG_HIP(hipGetDevice(&h->dev));
    // device address of the allocation-free solve's scratch, once per device
    (void)amg::noalloc_scratch(h->dev);
    amg::keep_pool_memory();
    amg::SetupStream on(h->stream, !h->own_stream);
    amg::PoolScope pool(h->stream);
    amg::build_hierarchy(h, A);
    amg::bootstrap_build(h);
    return AMG_OK;
  });
  for (amg_hierarchy *c : h->comp) c->stream = h->stream;
  h->p.smooth_vector = nullptr;
  h->p.model_params = nullptr;
  h->p.model_path = nullptr;
  if (st != AMG_OK) {
    std::string msg = g_last_error;
    amg_destroy(h);
    g_last_error = msg;
    return st;
  }
  *h_out = h;
  return AMG_OK;
}

int amg_pcg_solve(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
                  int32_t *iters_out, double *relres_out) {
  if (!h || !b || !x || !iters_out || !relres_out) return set_error(AMG_ERR_INVALID, "NULL argument");
  if (!(rtol > 0.0) || !std::isfinite(rtol) || maxit < 1)
    return set_error(AMG_ERR_INVALID, "rtol must be > 0 and maxit >= 1");
  return guarded([&] {
    int it = 0;
    double rel = 0.0;
    int st = amg::pcg_solve(h, b, x, rtol, maxit, &it, &rel);
    *iters_out = it;
    *relres_out = rel;
    if (st == AMG_ERR_NOT_SPD) g_last_error = "PCG breakdown: rho <= 0 (A or B not s.p.d.)";
    if (st == AMG_ERR_NONFINITE) g_last_error = "non-finite value in the iteration";
    return st;
  });
}

int amg_pcg_solve_noalloc(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
                          int32_t *iters_out, double *relres_out) {
  if (!h || !b || !x || !iters_out || !relres_out) return set_error(AMG_ERR_INVALID, "NULL argument");
  if (!(rtol > 0.0) || !std::isfinite(rtol) || maxit < 1)
    return set_error(AMG_ERR_INVALID, "rtol must be > 0 and maxit >= 1");
  return guarded([&] {
    int it = 0;
    double rel = 0.0;
    int st = amg::pcg_solve_noalloc(h, b, x, rtol, maxit, &it, &rel);
    *iters_out = it;
    *relres_out = rel;
    if (st == AMG_ERR_NOT_SPD) g_last_error = "PCG breakdown: rho <= 0 (A or B not s.p.d.)";
    if (st == AMG_ERR_NONFINITE) g_last_error = "non-finite value in the iteration";
    return st;
  });
}

int64_t amg_pcg_solve_noalloc_max_rows(void) { return amg::noalloc_max_rows(); }

void amg_destroy(amg_hierarchy *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  amg::destroy_graph(h);
  if (h->sc_host) (void)hipHostFree(h->sc_host);
  h->sc_host = nullptr;
  const bool own = h->own_stream;
  const int dev = h->stream_dev;
  hipStream_t s = h->stream;
  {
    amg::FreeOn on(amg::library_stream());   // h->stream is idle and may be the caller's
    amg::destroy_components(h);
    delete h;   // frees all device buffers
  }
  if (own) amg::release_private_stream(dev, s);
}

const char *amg_strerror(int code) {
  switch (code) {
    case AMG_OK: return "ok";
    case AMG_NOT_CONVERGED: return "not converged within maxit";
    case AMG_ERR_INVALID: return "invalid argument";
    case AMG_ERR_NOT_SPD: return "matrix or preconditioner not symmetric positive definite";
    case AMG_ERR_NONFINITE: return "non-finite value";
    case AMG_ERR_NOMEM: return "out of memory";
    case AMG_ERR_DEVICE: return "HIP device error";
    case AMG_ERR_UNSUPPORTED: return "unsupported parameter combination";
    case AMG_ERR_MODEL: return "learned smooth vector unusable (relaxation used instead)";
    default: return "unknown status";
  }
}

const char *amg_last_error(void) { return g_last_error.c_str(); }

int amg_info(const amg_hierarchy *h, amg_info_t *out) {
  if (!h || !out) return set_error(AMG_ERR_INVALID, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->levels = static_cast<int32_t>(h->L.size());
  double tot = 0.0;
  for (size_t k = 0; k < h->L.size(); ++k) {
    out->n[k] = h->L[k].A.n;
    out->nnz[k] = h->L[k].A.nnz;
    out->dict_size[k] = h->L[k].S.ndict;
    tot += static_cast<double>(h->L[k].A.nnz);
  }
  out->opc = tot / static_cast<double>(h->L[0].A.nnz);
  out->coarse_dense = h->coarse_dense;
  out->matching_rounds = h->tm.rounds;
  out->setup_ms = h->tm.setup_ms;
  out->setup_match_ms = h->tm.match_ms;
  out->setup_rap_ms = h->tm.rap_ms;
  out->setup_smooth_ms = h->tm.smooth_ms;
  out->device_bytes = amg::device_bytes(h);
  for (const amg_hierarchy *c : h->comp) out->device_bytes += amg::device_bytes(c) + c->ct.bytes() + c->ce.bytes();
  out->device_bytes += h->ct.bytes() + h->ce.bytes();
  out->nhrc = 1 + static_cast<int32_t>(h->comp.size());
  out->nrates = static_cast<int32_t>(std::min<size_t>(h->rates.size(), AMG_MAX_HRC));
  for (int j = 0; j < out->nrates; ++j) out->rates[j] = h->rates[j];
  out->setup_bootstrap_ms = h->tm.bootstrap_ms;
  out->smooth_status = h->smooth_status;
  return AMG_OK;
}

amg_hierarchy *amg_component(amg_hierarchy *h, int32_t j) {
  if (!h || j < 0 || j > static_cast<int32_t>(h->comp.size())) {
    set_error(AMG_ERR_INVALID, "no such hierarchy in the composite");
    return nullptr;
  }
  return j == 0 ? h : h->comp[j - 1];
}

int amg_export_level(const amg_hierarchy *h, int32_t k, int32_t *row_ptr, int32_t *col_idx,
                     double *val, double *dinv, double *w, int32_t *agg, double *pval) {
  if (!h) return set_error(AMG_ERR_INVALID, "NULL hierarchy");
  if (k < 0 || k >= static_cast<int32_t>(h->L.size())) return set_error(AMG_ERR_INVALID, "level out of range");
  return guarded([&] {
    const amg::Level &L = h->L[k];
    const auto d2h = hipMemcpyDeviceToHost;
    hipStream_t s = h->stream;
    if (row_ptr) AMG_HIP(hipMemcpyAsync(row_ptr, L.A.rp.p, sizeof(int) * (L.A.n + 1), d2h, s));
    if (col_idx) AMG_HIP(hipMemcpyAsync(col_idx, L.A.ci.p, sizeof(int) * L.A.nnz, d2h, s));
    if (val) AMG_HIP(hipMemcpyAsync(val, L.A.v.p, sizeof(double) * L.A.nnz, d2h, s));
    if (dinv) AMG_HIP(hipMemcpyAsync(dinv, L.dinv.p, sizeof(double) * L.A.n, d2h, s));
    if (w && L.w.p) AMG_HIP(hipMemcpyAsync(w, L.w.p, sizeof(double) * L.A.n, d2h, s));
    if (k + 1 < static_cast<int32_t>(h->L.size())) {
      if (agg) AMG_HIP(hipMemcpyAsync(agg, L.agg.p, sizeof(int) * L.A.n, d2h, s));
      if (pval) AMG_HIP(hipMemcpyAsync(pval, L.pval.p, sizeof(double) * L.A.n, d2h, s));
    }
    AMG_HIP(hipStreamSynchronize(s));
    return AMG_OK;
  });
}

int amg_vcycle(amg_hierarchy *h, const double *r, double *z) {
  if (!h || !r || !z || r == z) return set_error(AMG_ERR_INVALID, "bad argument");
  return guarded([&] {
    amg::enqueue_vcycle(h, r, z);
    return AMG_OK;
  });
}

int amg_spmv(amg_hierarchy *h, int32_t k, const double *x, double *y) {
  if (!h || !x || !y || x == y) return set_error(AMG_ERR_INVALID, "bad argument");
  if (k < 0 || k >= static_cast<int32_t>(h->L.size())) return set_error(AMG_ERR_INVALID, "level out of range");
  return guarded([&] {
    amg::enqueue_spmv(h, k, x, y);
    return AMG_OK;
  });
}

int amg_sweep(amg_hierarchy *h, int32_t k, const double *r, const double *x, double *xn) {
  if (!h || !r || !x || !xn || xn == x || xn == r) return set_error(AMG_ERR_INVALID, "bad argument");
  if (k < 0 || k >= static_cast<int32_t>(h->L.size())) return set_error(AMG_ERR_INVALID, "level out of range");
  return guarded([&] {
    amg::enqueue_sweep(h, k, r, x, xn);
    return AMG_OK;
  });
}

int amg_time_kernel(amg_hierarchy *h, int32_t kernel, int32_t k, int32_t reps, double *avg_ms,
                    double *bytes) {
  if (!h || !avg_ms || !bytes || reps < 1) return set_error(AMG_ERR_INVALID, "bad argument");
  return guarded([&] {
    amg::time_kernel(h, kernel, k, reps, avg_ms, bytes);
    return AMG_OK;
  });
}

}  // extern "C"
