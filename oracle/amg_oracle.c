/*
 * amg_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, obviously-correct CPU reference for the aggregation-AMG
 * preconditioned flexible CG of Bernaschi, Celestini, D'Ambra, Vella,
 * "Multi-GPU aggregation-based AMG preconditioner for iterative linear
 * solvers" (arXiv 2303.02352).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the GPU library never
 * links or calls it, and the two share no source.
 *
 * Arithmetic is IEEE binary64, compiled with -ffp-contract=off so that every
 * multiply and add rounds separately.  Every reduction is a left fold in
 * index order starting from +0.0 unless a function says otherwise.
 *
 * Paper sections followed:
 *   Sec. 3, Alg. 1 (flexible PCG)            -> orc_pcg
 *   Sec. 3.1, l1-Jacobi smoother             -> l1_dinv, sweep
 *   Sec. 3.1, Alg. 2 and the B^k operator    -> vcycle
 *   Sec. 3.1, Alg. 3 (coarsening by MWM),
 *             pairwise prolongators and
 *             their s-fold composition        -> orc_setup
 *   Sec. 4.1, Suitor 1/2-approximate MWM     -> orc_match_greedy, orc_match_suitor
 *   Sec. 5, operator complexity, stop rule   -> orc_opc, orc_pcg
 * Where the paper is silent the readings used are stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* CPU-baseline timing build only (compiled with -fopenmp; the parity build is
 * not): the row loops of SpMV, sweeps, residuals, prolongation and the PCG
 * vector updates run over static blocks of rows on all threads, and a dot
 * product folds each thread's block left to right, then the per-thread
 * partials in thread order.  Without OpenMP every loop below is the plain
 * sequential loop. */
#ifdef _OPENMP
#include <omp.h>
#define ORC_ROWS _Pragma("omp parallel for schedule(static)")
#else
#define ORC_ROWS
#endif

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_INVALID (-1)
#define ORC_NOT_SPD (-2)
#define ORC_NONFINITE (-3)
#define ORC_NOMEM (-4)

#define ORC_MAXLEV 64
#define ORC_DENSE_MAX 1024   /* largest coarsest level solved by dense Cholesky */
#define ORC_STAGNATION 0.95  /* stop coarsening when n_{k+1} > 0.95 n_k */

typedef struct {
  int32_t aggr_steps;    /* s: pairwise matching steps composed per level */
  int32_t max_levels;    /* hierarchy depth limit, fine level included */
  int32_t coarse_max;    /* stop coarsening once n <= coarse_max */
  int32_t coarse_solver; /* 0 dense Cholesky, 1 l1-Jacobi sweeps */
  int32_t coarse_sweeps; /* sweeps for coarse_solver 1 */
  int32_t pre_sweeps;
  int32_t post_sweeps;
  int32_t smooth_vec;    /* 0 ones, 1 relaxation from ones, 2 caller-given */
  int32_t smooth_sweeps; /* relaxation sweeps for smooth_vec 1 */
  int32_t precond;       /* 1 AMG V-cycle, 0 identity (plain CG) */
  int32_t n_parts;       /* decoupled aggregation: row blocks matched separately (>= 1) */
  int32_t cycle_type;    /* 0 V-cycle, 1 H-cycle, 2 W-cycle */
  int32_t relax_type;    /* smoother: 0 Jacobi, 1 forward/backward Gauss-Seidel,
                            3 symmetrized Gauss-Seidel, 4 l1-Jacobi */
  int32_t coarse_relax;  /* the same codes, for coarse_solver 1 */
  int32_t max_hrc;       /* bootstrap: most hierarchies in the composite (>= 1) */
  int32_t bootstrap_type;/* 0 multiplicative, 1 symmetrized multiplicative, 2 additive */
  int32_t bootstrap_its; /* iterations of the composite on A x = 0 per rate estimate */
  int32_t bootstrap_seed;/* seed of the random start vectors */
  double bootstrap_rate; /* desired convergence rate of the composite */
} orc_params;

typedef struct {
  int32_t n;
  int64_t nnz;
  int32_t *rp;
  int32_t *ci;
  double *v;
} csr_t;

#define ORC_MAXHRC 16

typedef struct orc_h orc_h;
struct orc_h {
  orc_params p;
  int nlev;
  csr_t A[ORC_MAXLEV];
  int32_t *part[ORC_MAXLEV]; /* row block (task) of each row, Sec. 4.1 */
  double *dinv[ORC_MAXLEV];
  double *w[ORC_MAXLEV];     /* smooth vector of each level */
  int32_t *agg[ORC_MAXLEV];  /* level k row -> level k+1 row */
  double *pval[ORC_MAXLEV];  /* the one nonzero of row i of P_k */
  int coarse_dense;          /* 1 if the coarsest level is solved directly */
  double *L;                 /* dense lower Cholesky factor, row-major */
  double *Ainv;              /* inverse of the coarsest matrix, row-major */
  /* V-cycle work vectors per level */
  double *vx[ORC_MAXLEV], *vt[ORC_MAXLEV], *vr[ORC_MAXLEV], *vres[ORC_MAXLEV], *ve[ORC_MAXLEV];
  double *vw[ORC_MAXLEV], *vz[ORC_MAXLEV];  /* second coarse correction (H/W cycles) */
  double *djac[ORC_MAXLEV];  /* 1 / a_ii (Jacobi and Gauss-Seidel smoothers) */
  /* binary32 copies for the mixed-precision V-cycle (built on first use) */
  float *fv[ORC_MAXLEV], *fdinv[ORC_MAXLEV], *fpval[ORC_MAXLEV];
  float *fx[ORC_MAXLEV], *ft[ORC_MAXLEV], *fr[ORC_MAXLEV], *fres[ORC_MAXLEV], *fe[ORC_MAXLEV];
  int have_f32;
  /* bootstrap composite: hierarchies 2..nhrc (hierarchy 1 is this one) and
   * the rate estimates (rate[j-1]: composite of the first j hierarchies) */
  int nhrc;
  orc_h *hrc[ORC_MAXHRC];
  double rate[ORC_MAXHRC];
  int nrate;
};

/* ------------------------------------------------------------------ utils */

static void csr_free(csr_t *a) {
  free(a->rp); free(a->ci); free(a->v);
  a->rp = NULL; a->ci = NULL; a->v = NULL; a->n = 0; a->nnz = 0;
}

static int csr_alloc(csr_t *a, int32_t n, int64_t nnz) {
  a->n = n; a->nnz = nnz;
  a->rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  a->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  a->v = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  if (!a->rp || !a->ci || !a->v) { csr_free(a); return ORC_NOMEM; }
  return ORC_OK;
}

/* Structural and numerical checks on the input: sorted in-range columns,
 * present positive diagonal, finite values, bitwise symmetry (the method is
 * defined for s.p.d. A, Sec. 1 and 3). */
int orc_validate(int32_t n, const int32_t *rp, const int32_t *ci, const double *v) {
  if (n <= 0 || !rp || !ci || !v) return ORC_INVALID;
  if (rp[0] != 0) return ORC_INVALID;
  for (int32_t i = 0; i < n; i++) {
    if (rp[i + 1] < rp[i]) return ORC_INVALID;
    int has_diag = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
      if (ci[k] < 0 || ci[k] >= n) return ORC_INVALID;
      if (k > rp[i] && ci[k] <= ci[k - 1]) return ORC_INVALID;
      if (!isfinite(v[k])) return ORC_NONFINITE;
      if (ci[k] == i) {
        has_diag = 1;
        if (!(v[k] > 0.0)) return ORC_NOT_SPD;
      }
    }
    if (!has_diag) return ORC_NOT_SPD;
  }
  /* symmetry: a_ij must equal a_ji bit for bit */
  for (int32_t i = 0; i < n; i++) {
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
      int32_t j = ci[k];
      int found = 0;
      for (int32_t m = rp[j]; m < rp[j + 1]; m++) {
        if (ci[m] == i) {
          found = (memcmp(&v[m], &v[k], sizeof(double)) == 0);
          break;
        }
      }
      if (!found) return ORC_INVALID;
    }
  }
  return ORC_OK;
}

/* y = A x, each row a left fold of a_ij * x_j in CSR order from +0.0. */
static void spmv(const csr_t *A, const double *x, double *y) {
  ORC_ROWS
  for (int32_t i = 0; i < A->n; i++) {
    double s = 0.0;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) s = s + A->v[k] * x[A->ci[k]];
    y[i] = s;
  }
}

int orc_spmv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
             const double *x, double *y) {
  csr_t A = {n, rp[n], (int32_t *)rp, (int32_t *)ci, (double *)v};
  spmv(&A, x, y);
  return ORC_OK;
}

static double dot(int32_t n, const double *a, const double *b) {
#ifdef _OPENMP
  double part[1024];
  int nt = omp_get_max_threads();
  if (nt > 1024) nt = 1024;
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num(), m = omp_get_num_threads();
    int64_t lo = (int64_t)n * t / m, hi = (int64_t)n * (t + 1) / m;
    double s = 0.0;
    for (int64_t i = lo; i < hi; i++) s = s + a[i] * b[i];
    part[t] = s;
    if (t == 0) nt = m;
  }
  double s = 0.0;
  for (int t = 0; t < nt; t++) s = s + part[t];
  return s;
#else
  double s = 0.0;
  for (int32_t i = 0; i < n; i++) s = s + a[i] * b[i];
  return s;
#endif
}

/* l1-Jacobi (Sec. 3.1): M_ii = a_ii + sum_{j != i} |a_ij|.  The printed
 * formula lacks the absolute value; without it every interior Poisson row
 * gives M_ii = 0, so the l1 form (absolute values) is used.  Computed as the
 * left fold of |a_ij| over the whole row in CSR order; dinv = 1 / M_ii. */
static void l1_dinv(const csr_t *A, double *dinv) {
  for (int32_t i = 0; i < A->n; i++) {
    double m = 0.0;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) m = m + fabs(A->v[k]);
    dinv[i] = 1.0 / m;
  }
}

int orc_l1_dinv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, double *dinv) {
  csr_t A = {n, rp[n], (int32_t *)rp, (int32_t *)ci, (double *)v};
  l1_dinv(&A, dinv);
  return ORC_OK;
}

/* One l1-Jacobi sweep: xn = x + dinv * (r - A x).  xn must not alias x. */
static void sweep(const csr_t *A, const double *dinv, const double *r, const double *x, double *xn) {
  ORC_ROWS
  for (int32_t i = 0; i < A->n; i++) {
    double s = 0.0;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) s = s + A->v[k] * x[A->ci[k]];
    xn[i] = x[i] + dinv[i] * (r[i] - s);
  }
}

/* ------------------------------------------------------ matching weights */

/* Edge weight of the matching graph.  Sec. 3.1 leaves the function of the
 * smooth vector and the matrix entries unspecified; the one of the compatible
 * weighted matching papers it cites is used:
 *   w_hat_ij = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2),
 * evaluated with i = min, j = max of the pair so both ends get the same bits:
 *   num = ((2 a_ij) w_i) w_j,  den = (a_ii w_i) w_i + (a_jj w_j) w_j.       */
static double edge_weight(double aij, double aii, double ajj, double wi, double wj) {
  double num = ((2.0 * aij) * wi) * wj;
  double den = (aii * wi) * wi + (ajj * wj) * wj;
  return 1.0 - num / den;
}

static double *diag_of(const csr_t *A) {
  double *d = (double *)malloc(sizeof(double) * (size_t)A->n);
  if (!d) return NULL;
  for (int32_t i = 0; i < A->n; i++) {
    d[i] = 0.0;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++)
      if (A->ci[k] == i) d[i] = A->v[k];
  }
  return d;
}

/* Weight of every stored entry (diagonal slots get NaN).  Exposed for tests. */
int orc_edge_weights(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                     const double *w, double *out) {
  csr_t A = {n, rp[n], (int32_t *)rp, (int32_t *)ci, (double *)v};
  double *d = diag_of(&A);
  if (!d) return ORC_NOMEM;
  for (int32_t i = 0; i < n; i++)
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
      int32_t j = ci[k];
      if (j == i) { out[k] = NAN; continue; }
      int32_t lo = i < j ? i : j, hi = i < j ? j : i;
      out[k] = edge_weight(v[k], d[lo], d[hi], w[lo], w[hi]);
    }
  free(d);
  return ORC_OK;
}

/* ---------------------------------------------------------------- matching
 * Sec. 4.1 uses Suitor, a 1/2-approximate maximum weight matching.  Suitor
 * names no tie rule; edges are totally ordered by the key
 *   (weight, max(i,j), min(i,j))   compared lexicographically, larger wins,
 * and an edge is eligible when a_ij != 0 and its weight is > 0.  Under a
 * strict total order Suitor, the locally-dominant algorithm and sequential
 * greedy all return the same matching; the greedy form below is the oracle
 * and the Suitor form is kept to show that equality in tests.              */

typedef struct { double w; int32_t hi, lo; } edge_t;

static int key_greater(double wa, int32_t ha, int32_t la, double wb, int32_t hb, int32_t lb) {
  if (wa != wb) return wa > wb;
  if (ha != hb) return ha > hb;
  return la > lb;
}

static int edge_cmp_desc(const void *pa, const void *pb) {
  const edge_t *a = (const edge_t *)pa, *b = (const edge_t *)pb;
  if (key_greater(a->w, a->hi, a->lo, b->w, b->hi, b->lo)) return -1;
  if (key_greater(b->w, b->hi, b->lo, a->w, a->hi, a->lo)) return 1;
  return 0;
}

/* Sequential greedy: scan eligible edges by decreasing key, match when both
 * ends are free.  mate[i] = partner or -1.  With part != NULL (decoupled
 * aggregation, Sec. 4.1) an edge whose ends lie in different row blocks is
 * not eligible: each block is matched as its own local subgraph. */
static int match_greedy(const csr_t *A, const double *w, const int32_t *part, int32_t *mate) {
  double *d = diag_of(A);
  if (!d) return ORC_NOMEM;
  int64_t m = 0;
  for (int32_t i = 0; i < A->n; i++)
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++)
      if (A->ci[k] > i) m++;
  edge_t *E = (edge_t *)malloc(sizeof(edge_t) * (size_t)(m > 0 ? m : 1));
  if (!E) { free(d); return ORC_NOMEM; }
  int64_t e = 0;
  for (int32_t i = 0; i < A->n; i++)
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) {
      int32_t j = A->ci[k];
      if (j <= i || A->v[k] == 0.0) continue;
      if (part && part[i] != part[j]) continue;
      double wt = edge_weight(A->v[k], d[i], d[j], w[i], w[j]);
      if (!(wt > 0.0)) continue;
      E[e].w = wt; E[e].hi = j; E[e].lo = i; e++;
    }
  qsort(E, (size_t)e, sizeof(edge_t), edge_cmp_desc);
  for (int32_t i = 0; i < A->n; i++) mate[i] = -1;
  for (int64_t t = 0; t < e; t++) {
    if (mate[E[t].hi] < 0 && mate[E[t].lo] < 0) {
      mate[E[t].hi] = E[t].lo;
      mate[E[t].lo] = E[t].hi;
    }
  }
  free(E); free(d);
  return ORC_OK;
}

int orc_match_greedy(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                     const double *w, int32_t *mate) {
  csr_t A = {n, rp[n], (int32_t *)rp, (int32_t *)ci, (double *)v};
  return match_greedy(&A, w, NULL, mate);
}

/* ------------------------------------------------- decoupled aggregation
 * Sec. 4.1: every task owns a block of consecutive rows and matches only the
 * subgraph of its own rows.  Block p of n rows split into np blocks is
 * [floor(p n / np), floor((p+1) n / np)).  An aggregate then lies inside one
 * block, and the coarse row it becomes belongs to that block; since
 * aggregates are numbered by their smallest row, the coarse blocks are again
 * consecutive ranges. */
static void row_blocks(int32_t n, int32_t np, int32_t *part) {
  for (int32_t p = 0; p < np; p++) {
    int64_t a = (int64_t)p * n / np, b = (int64_t)(p + 1) * n / np;
    for (int64_t i = a; i < b; i++) part[i] = p;
  }
}

int orc_row_blocks(int32_t n, int32_t np, int32_t *part) {
  if (n < 1 || np < 1) return ORC_INVALID;
  row_blocks(n, np, part);
  return ORC_OK;
}

/* Sequential Suitor (Manne and Halappanavar): each vertex proposes to its
 * heaviest neighbour whose current suitor it beats; a displaced suitor
 * proposes again.  Vertices start in the caller's order.  Independent of
 * match_greedy; tests check that both give the same mate[]. */
int orc_match_suitor(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                     const double *w, const int32_t *order, int32_t *mate) {
  csr_t A = {n, rp[n], (int32_t *)rp, (int32_t *)ci, (double *)v};
  double *d = diag_of(&A);
  int32_t *suitor = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  double *ws = (double *)malloc(sizeof(double) * (size_t)n);
  if (!d || !suitor || !ws) { free(d); free(suitor); free(ws); return ORC_NOMEM; }
  for (int32_t i = 0; i < n; i++) { suitor[i] = -1; ws[i] = 0.0; }
  for (int32_t t = 0; t < n; t++) {
    int32_t cur = order[t];
    while (cur >= 0) {
      int32_t best = -1; double bw = 0.0;
      for (int32_t k = rp[cur]; k < rp[cur + 1]; k++) {
        int32_t u = ci[k];
        if (u == cur || v[k] == 0.0) continue;
        int32_t lo = cur < u ? cur : u, hi = cur < u ? u : cur;
        double wt = edge_weight(v[k], d[lo], d[hi], w[lo], w[hi]);
        if (!(wt > 0.0)) continue;
        /* must beat u's current suitor edge (suitor[u], u) */
        if (suitor[u] >= 0) {
          int32_t s = suitor[u];
          int32_t slo = s < u ? s : u, shi = s < u ? u : s;
          if (!key_greater(wt, hi, lo, ws[u], shi, slo)) continue;
        }
        if (best < 0) { best = u; bw = wt; continue; }
        int32_t blo = cur < best ? cur : best, bhi = cur < best ? best : cur;
        if (key_greater(wt, hi, lo, bw, bhi, blo)) { best = u; bw = wt; }
      }
      if (best < 0) break;
      int32_t prev = suitor[best];
      suitor[best] = cur;
      ws[best] = bw;
      cur = prev;
    }
  }
  for (int32_t i = 0; i < n; i++) {
    int32_t s = suitor[i];
    mate[i] = (s >= 0 && suitor[s] == i) ? s : -1;
  }
  free(d); free(suitor); free(ws);
  return ORC_OK;
}

/* ------------------------------------------------- aggregates and P values */

/* Coarse numbering (silent in the paper): aggregates are numbered by their
 * smallest fine index, ascending.  Returns the number of aggregates. */
static int32_t aggregate_ids(int32_t n, const int32_t *mate, int32_t *agg) {
  int32_t c = 0;
  for (int32_t i = 0; i < n; i++) agg[i] = -1;
  for (int32_t i = 0; i < n; i++) {
    if (agg[i] >= 0) continue;
    agg[i] = c;
    if (mate[i] >= 0) agg[mate[i]] = c;
    c++;
  }
  return c;
}

/* Pairwise prolongator values (Sec. 3.1: one nonzero per row, values taken
 * from the smooth vector): p_m = w_m / ||w restricted to the aggregate||,
 * norm = sqrt(w_a^2 + w_b^2) over members in ascending order; a singleton
 * with w_i = 0 gets p = 1.  Then w_c = P^T w, folded over members ascending. */
static void pair_pvals(int32_t n, const int32_t *mate, const double *w, double *p) {
  for (int32_t i = 0; i < n; i++) {
    int32_t j = mate[i];
    double nrm;
    if (j < 0) {                      /* singleton: p = w_i / |w_i| = +-1 */
      p[i] = (w[i] == 0.0) ? 1.0 : w[i] / fabs(w[i]);
      continue;
    }
    int32_t lo = i < j ? i : j, hi = i < j ? j : i;
    nrm = sqrt(w[lo] * w[lo] + w[hi] * w[hi]);
    p[i] = w[i] / nrm;
  }
}

static void restrict_fold(int32_t n, int32_t nc, const int32_t *agg, const double *p,
                          const double *x, double *xc) {
  /* members of each aggregate visited in ascending fine index */
  for (int32_t I = 0; I < nc; I++) xc[I] = 0.0;
  for (int32_t i = 0; i < n; i++) xc[agg[i]] = xc[agg[i]] + p[i] * x[i];
}

/* ------------------------------------------------------- Galerkin product
 * A_c = P^T A P (Sec. 3.1, Alg. 3).  With one nonzero per row of P,
 *   A_c(I,J) = sum over stored a_ij with agg(i)=I, agg(j)=J of (p_i p_j) a_ij.
 * Summation order (silent in the paper): the terms of entry (I,J) are folded
 * in ascending (u, v), where u is the fine index on the side of min(I,J) and
 * v the other one.  Entry (J,I) then sees the same terms in the same order,
 * so a bitwise-symmetric A gives a bitwise-symmetric A_c.  Entries that
 * cancel to zero are kept. */
typedef struct { int32_t J, u, v; double t; } term_t;

static int term_cmp(const void *pa, const void *pb) {
  const term_t *a = (const term_t *)pa, *b = (const term_t *)pb;
  if (a->J != b->J) return a->J < b->J ? -1 : 1;
  if (a->u != b->u) return a->u < b->u ? -1 : 1;
  if (a->v != b->v) return a->v < b->v ? -1 : 1;
  return 0;
}

static int galerkin(const csr_t *A, int32_t nc, const int32_t *agg, const double *p, csr_t *Ac) {
  int32_t n = A->n;
  /* members of each aggregate, ascending */
  int32_t *mp = (int32_t *)calloc((size_t)nc + 1, sizeof(int32_t));
  int32_t *mem = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
  if (!mp || !mem || !fill) { free(mp); free(mem); free(fill); return ORC_NOMEM; }
  for (int32_t i = 0; i < n; i++) mp[agg[i] + 1]++;
  for (int32_t I = 0; I < nc; I++) mp[I + 1] += mp[I];
  for (int32_t I = 0; I < nc; I++) fill[I] = mp[I];
  for (int32_t i = 0; i < n; i++) mem[fill[agg[i]]++] = i;
  free(fill);

  /* first pass over rows to size the term buffer and the output */
  int64_t maxterms = 0;
  for (int32_t I = 0; I < nc; I++) {
    int64_t c = 0;
    for (int32_t m = mp[I]; m < mp[I + 1]; m++) c += A->rp[mem[m] + 1] - A->rp[mem[m]];
    if (c > maxterms) maxterms = c;
  }
  term_t *T = (term_t *)malloc(sizeof(term_t) * (size_t)(maxterms > 0 ? maxterms : 1));
  int64_t cap = A->nnz > 0 ? A->nnz : 1;
  int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  double *cv = (double *)malloc(sizeof(double) * (size_t)cap);
  int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
  if (!T || !ci || !cv || !rp) {
    free(T); free(ci); free(cv); free(rp); free(mp); free(mem); return ORC_NOMEM;
  }
  int64_t out = 0;
  rp[0] = 0;
  for (int32_t I = 0; I < nc; I++) {
    int64_t c = 0;
    for (int32_t m = mp[I]; m < mp[I + 1]; m++) {
      int32_t i = mem[m];
      for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) {
        int32_t j = A->ci[k];
        int32_t J = agg[j];
        T[c].J = J;
        if (I <= J) { T[c].u = i; T[c].v = j; } else { T[c].u = j; T[c].v = i; }
        T[c].t = (p[i] * p[j]) * A->v[k];
        c++;
      }
    }
    qsort(T, (size_t)c, sizeof(term_t), term_cmp);
    for (int64_t t = 0; t < c;) {
      double s = T[t].t;
      int64_t q = t + 1;
      while (q < c && T[q].J == T[t].J) { s = s + T[q].t; q++; }
      ci[out] = T[t].J; cv[out] = s; out++;
      t = q;
    }
    rp[I + 1] = (int32_t)out;
  }
  free(T); free(mp); free(mem);
  Ac->n = nc; Ac->nnz = out; Ac->rp = rp;
  Ac->ci = (int32_t *)realloc(ci, sizeof(int32_t) * (size_t)(out > 0 ? out : 1));
  Ac->v = (double *)realloc(cv, sizeof(double) * (size_t)(out > 0 ? out : 1));
  return ORC_OK;
}

/* ------------------------------------------------------ dense coarsest solve
 * The coarsest system is solved directly (Alg. 2); Cholesky A = L L^T.
 * L_jj = sqrt(a_jj - sum_{k<j} L_jk^2), L_ij = (a_ij - sum_{k<j} L_ik L_jk)/L_jj,
 * sums folded with k ascending.  A pivot <= 0 means A is not s.p.d.        */
static int cholesky(int32_t n, const double *A, double *L) {
  for (int64_t t = 0; t < (int64_t)n * n; t++) L[t] = 0.0;
  for (int32_t j = 0; j < n; j++) {
    double s = A[(int64_t)j * n + j];
    for (int32_t k = 0; k < j; k++) s = s - L[(int64_t)j * n + k] * L[(int64_t)j * n + k];
    if (!(s > 0.0)) return ORC_NOT_SPD;
    double ljj = sqrt(s);
    L[(int64_t)j * n + j] = ljj;
    for (int32_t i = j + 1; i < n; i++) {
      double t = A[(int64_t)i * n + j];
      for (int32_t k = 0; k < j; k++) t = t - L[(int64_t)i * n + k] * L[(int64_t)j * n + k];
      L[(int64_t)i * n + j] = t / ljj;
    }
  }
  return ORC_OK;
}

/* L y = r (k ascending), then L^T x = y (k descending). */
static void chol_solve(int32_t n, const double *L, const double *r, double *x) {
  for (int32_t i = 0; i < n; i++) {
    double s = r[i];
    for (int32_t k = 0; k < i; k++) s = s - L[(int64_t)i * n + k] * x[k];
    x[i] = s / L[(int64_t)i * n + i];
  }
  for (int32_t i = n - 1; i >= 0; i--) {
    double s = x[i];
    for (int32_t k = n - 1; k > i; k--) s = s - L[(int64_t)k * n + i] * x[k];
    x[i] = s / L[(int64_t)i * n + i];
  }
}

int orc_cholesky(int32_t n, const double *A, double *L) { return cholesky(n, A, L); }
int orc_chol_solve(int32_t n, const double *L, const double *r, double *x) {
  chol_solve(n, L, r, x);
  return ORC_OK;
}

/* ----------------------------------------------------------------- setup */

void orc_free(orc_h *h);

static int smooth_vector(const orc_params *p, const csr_t *A, const double *dinv,
                         const double *given, double *w) {
  int32_t n = A->n;
  if (p->smooth_vec == 2) {
    if (!given) return ORC_INVALID;
    for (int32_t i = 0; i < n; i++) {
      if (!isfinite(given[i])) return ORC_NONFINITE;
      w[i] = given[i];
    }
    return ORC_OK;
  }
  for (int32_t i = 0; i < n; i++) w[i] = 1.0;
  if (p->smooth_vec == 0) return ORC_OK;
  /* relaxation on A w = 0 from w = 1, then scale by max |w| */
  double *z = (double *)calloc((size_t)n, sizeof(double));
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  if (!z || !t) { free(z); free(t); return ORC_NOMEM; }
  for (int32_t s = 0; s < p->smooth_sweeps; s++) {
    sweep(A, dinv, z, w, t);
    memcpy(w, t, sizeof(double) * (size_t)n);
  }
  /* a non-finite or all-zero result falls back to the constant vector */
  double mx = 0.0;
  int finite = 1;
  for (int32_t i = 0; i < n; i++) {
    if (!isfinite(w[i])) finite = 0;
    else if (fabs(w[i]) > mx) mx = fabs(w[i]);
  }
  if (finite && mx > 0.0) {
    for (int32_t i = 0; i < n; i++) w[i] = w[i] / mx;
  } else {
    for (int32_t i = 0; i < n; i++) w[i] = 1.0;
  }
  free(z); free(t);
  return ORC_OK;
}

/* Alg. 3 with the s-step composition of Sec. 3.1.  Per level: s pairwise
 * steps (match, aggregate, P values, w_c = P^T w, A_c = P^T A P), stopping
 * early once n <= coarse_max; the composite P has aggregate map
 * agg = agg_s(...agg_1) and value p = p_1 * p_2(agg_1) * ...; the coarse
 * matrix is the last pairwise A_c (equal to the composite Galerkin product
 * in exact arithmetic).  Coarsening stops at n <= coarse_max, at max_levels,
 * or when a level shrinks by less than 5%. */
static orc_h *build_single(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                           const orc_params *par, const double *w_given, int *status) {
  *status = orc_validate(n, rp, ci, v);
  if (*status != ORC_OK) return NULL;
  if (par->aggr_steps < 1 || par->max_levels < 1 || par->coarse_max < 1 ||
      par->pre_sweeps < 0 || par->post_sweeps < 0 || par->coarse_sweeps < 1 ||
      par->smooth_sweeps < 0 || par->n_parts < 1) {
    *status = ORC_INVALID; return NULL;
  }
  if (par->max_hrc < 1 || par->max_hrc > ORC_MAXHRC || par->bootstrap_type < 0 ||
      par->bootstrap_type > 2 || par->bootstrap_its < 1 ||
      !(par->bootstrap_rate > 0.0 && par->bootstrap_rate <= 1.0)) {
    *status = ORC_INVALID; return NULL;
  }
  if (par->cycle_type < 0 || par->cycle_type > 2) { *status = ORC_INVALID; return NULL; }
  for (int q = 0; q < 2; q++) {
    int t = q ? par->coarse_relax : par->relax_type;
    if (t != 0 && t != 1 && t != 3 && t != 4) { *status = ORC_INVALID; return NULL; }
  }
  orc_h *h = (orc_h *)calloc(1, sizeof(orc_h));
  if (!h) { *status = ORC_NOMEM; return NULL; }
  h->p = *par;
  if (csr_alloc(&h->A[0], n, rp[n]) != ORC_OK) { free(h); *status = ORC_NOMEM; return NULL; }
  memcpy(h->A[0].rp, rp, sizeof(int32_t) * (size_t)(n + 1));
  memcpy(h->A[0].ci, ci, sizeof(int32_t) * (size_t)rp[n]);
  memcpy(h->A[0].v, v, sizeof(double) * (size_t)rp[n]);
  h->nlev = 1;
  h->dinv[0] = (double *)malloc(sizeof(double) * (size_t)n);
  h->w[0] = (double *)malloc(sizeof(double) * (size_t)n);
  if (!h->dinv[0] || !h->w[0]) { orc_free(h); *status = ORC_NOMEM; return NULL; }
  l1_dinv(&h->A[0], h->dinv[0]);
  *status = smooth_vector(par, &h->A[0], h->dinv[0], w_given, h->w[0]);
  if (*status != ORC_OK) { orc_free(h); return NULL; }
  h->part[0] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!h->part[0]) { orc_free(h); *status = ORC_NOMEM; return NULL; }
  row_blocks(n, par->n_parts, h->part[0]);

  int maxlev = par->max_levels < ORC_MAXLEV ? par->max_levels : ORC_MAXLEV;
  while (par->precond && h->nlev < maxlev && h->A[h->nlev - 1].n > par->coarse_max) {
    int k = h->nlev - 1;
    int32_t nk = h->A[k].n;
    csr_t cur = h->A[k];       /* borrowed for step 0 */
    double *wcur = h->w[k];
    int32_t *pcur = h->part[k];
    int32_t *aggt = (int32_t *)malloc(sizeof(int32_t) * (size_t)nk);
    double *pt = (double *)malloc(sizeof(double) * (size_t)nk);
    if (!aggt || !pt) { free(aggt); free(pt); orc_free(h); *status = ORC_NOMEM; return NULL; }
    for (int32_t i = 0; i < nk; i++) { aggt[i] = i; pt[i] = 1.0; }
    int owned = 0;
    for (int step = 0; step < par->aggr_steps; step++) {
      if (step > 0 && cur.n <= par->coarse_max) break;
      int32_t m = cur.n;
      int32_t *mate = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
      int32_t *a1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
      double *p1 = (double *)malloc(sizeof(double) * (size_t)m);
      if (!mate || !a1 || !p1) { *status = ORC_NOMEM; }
      else *status = match_greedy(&cur, wcur, pcur, mate);
      if (*status != ORC_OK) {
        free(mate); free(a1); free(p1); free(aggt); free(pt);
        if (owned) { csr_free(&cur); free(wcur); free(pcur); }
        orc_free(h); return NULL;
      }
      int32_t mc = aggregate_ids(m, mate, a1);
      pair_pvals(m, mate, wcur, p1);
      double *wc = (double *)malloc(sizeof(double) * (size_t)mc);
      int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(mc > 0 ? mc : 1));
      csr_t Ac;
      memset(&Ac, 0, sizeof(Ac));
      *status = (wc && pc) ? galerkin(&cur, mc, a1, p1, &Ac) : ORC_NOMEM;
      if (*status != ORC_OK) {
        free(mate); free(a1); free(p1); free(wc); free(pc); free(aggt); free(pt);
        if (owned) { csr_free(&cur); free(wcur); free(pcur); }
        orc_free(h); return NULL;
      }
      restrict_fold(m, mc, a1, p1, wcur, wc);
      /* the coarse row of an aggregate stays in its members' block */
      for (int32_t i = 0; i < m; i++) pc[a1[i]] = pcur[i];
      for (int32_t i = 0; i < nk; i++) {
        pt[i] = pt[i] * p1[aggt[i]];
        aggt[i] = a1[aggt[i]];
      }
      if (owned) { csr_free(&cur); free(wcur); free(pcur); }
      cur = Ac; wcur = wc; pcur = pc; owned = 1;
      free(mate); free(a1); free(p1);
    }
    if (!owned || (double)cur.n > ORC_STAGNATION * (double)nk) {
      if (owned) { csr_free(&cur); free(wcur); free(pcur); }
      free(aggt); free(pt);
      break;
    }
    h->agg[k] = aggt; h->pval[k] = pt;
    h->A[k + 1] = cur; h->w[k + 1] = wcur; h->part[k + 1] = pcur;
    h->dinv[k + 1] = (double *)malloc(sizeof(double) * (size_t)cur.n);
    if (!h->dinv[k + 1]) { h->nlev = k + 2; orc_free(h); *status = ORC_NOMEM; return NULL; }
    l1_dinv(&h->A[k + 1], h->dinv[k + 1]);
    h->nlev = k + 2;
  }
  /* coarsest level solver */
  const csr_t *C = &h->A[h->nlev - 1];
  h->coarse_dense = par->precond && par->coarse_solver == 0 && C->n <= ORC_DENSE_MAX && h->nlev > 0;
  if (h->coarse_dense) {
    int32_t m = C->n;
    double *D = (double *)calloc((size_t)m * m, sizeof(double));
    h->L = (double *)malloc(sizeof(double) * (size_t)m * m);
    if (!D || !h->L) { free(D); orc_free(h); *status = ORC_NOMEM; return NULL; }
    for (int32_t i = 0; i < m; i++)
      for (int32_t k = C->rp[i]; k < C->rp[i + 1]; k++) D[(int64_t)i * m + C->ci[k]] = C->v[k];
    *status = cholesky(m, D, h->L);
    free(D);
    if (*status != ORC_OK) { orc_free(h); return NULL; }
    /* the direct solve z = A^-1 r uses the inverse, column j = chol_solve(e_j) */
    h->Ainv = (double *)malloc(sizeof(double) * (size_t)m * m);
    double *e = (double *)calloc((size_t)m, sizeof(double));
    double *col = (double *)malloc(sizeof(double) * (size_t)m);
    if (!h->Ainv || !e || !col) { free(e); free(col); orc_free(h); *status = ORC_NOMEM; return NULL; }
    for (int32_t j = 0; j < m; j++) {
      e[j] = 1.0;
      chol_solve(m, h->L, e, col);
      e[j] = 0.0;
      for (int32_t i = 0; i < m; i++) h->Ainv[(int64_t)i * m + j] = col[i];
    }
    free(e); free(col);
  }
  for (int k = 0; k < h->nlev; k++) {
    size_t nb = sizeof(double) * (size_t)h->A[k].n;
    h->vx[k] = (double *)malloc(nb); h->vt[k] = (double *)malloc(nb);
    h->vr[k] = (double *)malloc(nb); h->vres[k] = (double *)malloc(nb);
    h->ve[k] = (double *)malloc(nb);
    h->vw[k] = (double *)malloc(nb); h->vz[k] = (double *)malloc(nb);
    h->djac[k] = (double *)malloc(nb);
    if (!h->vx[k] || !h->vt[k] || !h->vr[k] || !h->vres[k] || !h->ve[k] || !h->vw[k] || !h->vz[k] ||
        !h->djac[k]) {
      orc_free(h); *status = ORC_NOMEM; return NULL;
    }
    /* Jacobi / Gauss-Seidel diagonal: 1 / a_ii */
    const csr_t *Ak = &h->A[k];
    for (int32_t i = 0; i < Ak->n; i++) {
      double d = 0.0;
      for (int32_t t = Ak->rp[i]; t < Ak->rp[i + 1]; t++)
        if (Ak->ci[t] == i) d = Ak->v[t];
      h->djac[k][i] = 1.0 / d;
    }
  }
  *status = ORC_OK;
  return h;
}

void orc_free(orc_h *h) {
  if (!h) return;
  for (int j = 0; j < ORC_MAXHRC; j++) orc_free(h->hrc[j]);
  for (int k = 0; k < ORC_MAXLEV; k++) {
    csr_free(&h->A[k]);
    free(h->dinv[k]); free(h->w[k]); free(h->agg[k]); free(h->pval[k]); free(h->part[k]);
    free(h->vx[k]); free(h->vt[k]); free(h->vr[k]); free(h->vres[k]); free(h->ve[k]);
    free(h->vw[k]); free(h->vz[k]); free(h->djac[k]);
    free(h->fv[k]); free(h->fdinv[k]); free(h->fpval[k]);
    free(h->fx[k]); free(h->ft[k]); free(h->fr[k]); free(h->fres[k]); free(h->fe[k]);
  }
  free(h->L);
  free(h->Ainv);
  free(h);
}

/* ---------------------------------------------------------------- V-cycle
 * Alg. 2 as the operator B^k it defines: with S the nu-sweep l1-Jacobi
 * operator started from zero,
 *   x  = S_pre(r)
 *   x += P_k Vcycle(k+1, P_k^T (r - A_k x))
 *   x  = x + dinv (r - A_k x), post_sweeps times
 * and at the coarsest level the Cholesky solve (or coarse_sweeps sweeps).
 * Writes the result into z (length n_k). */
static void smooth_from_zero(const csr_t *A, const double *dinv, const double *r, int nsw,
                             double *x, double *t) {
  int32_t n = A->n;
  if (nsw <= 0) { for (int32_t i = 0; i < n; i++) x[i] = 0.0; return; }
  ORC_ROWS
  for (int32_t i = 0; i < n; i++) x[i] = dinv[i] * r[i];
  for (int s = 1; s < nsw; s++) {
    sweep(A, dinv, r, x, t);
    memcpy(x, t, sizeof(double) * (size_t)n);
  }
}

/* Coarsest direct solve z = (A^nl)^-1 r (Alg. 2): row i of the inverse
 * times r, folded over j ascending. */
static void coarse_direct(const orc_h *h, const double *r, double *z) {
  int32_t n = h->A[h->nlev - 1].n;
  for (int32_t i = 0; i < n; i++) {
    double s = 0.0;
    for (int32_t j = 0; j < n; j++) s = s + h->Ainv[(int64_t)i * n + j] * r[j];
    z[i] = s;
  }
}

/* ---------------------------------------------- smoothers (Appendix A)
 * relax_type / coarse_relax codes:
 *   4 l1-Jacobi  x <- x + M^-1 (r - A x), M_ii = sum_j |a_ij| (Sec. 3.1);
 *   0 Jacobi     the same with a_ii;
 *   1 FGS/BGS    Gauss-Seidel: forward (rows ascending) before the coarse
 *                correction, backward (rows descending) after it, so that
 *                the cycle stays symmetric;
 *   3 symmetrized Gauss-Seidel: every sweep a forward then a backward pass.
 * A Gauss-Seidel pass updates row by row in place,
 *   x_i <- x_i + (r_i - sum_j a_ij x_j) / a_ii,
 * the row folded in CSR order over the current x.  Smoothing from zero:
 * the Jacobi types start with x = dinv r and do nsw - 1 further sweeps; the
 * Gauss-Seidel types start from x = 0 and do nsw sweeps. */
static void gs_pass(const csr_t *A, const double *dj, const double *r, double *x, int forward) {
  int32_t n = A->n;
  for (int32_t q = 0; q < n; q++) {
    int32_t i = forward ? q : n - 1 - q;
    double s = 0.0;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) s = s + A->v[k] * x[A->ci[k]];
    x[i] = x[i] + dj[i] * (r[i] - s);
  }
}

/* nsw sweeps of smoother `type` on A_k x = r continuing from x; pass = +1
 * pre-smoothing, -1 post-smoothing, 0 coarsest level (for FGS/BGS: forward
 * and backward passes alternate there, starting forward). */
static void smooth_more(orc_h *h, int k, int type, int pass, const double *r, int nsw, double *x) {
  const csr_t *A = &h->A[k];
  double *t = h->vt[k];
  for (int q = 0; q < nsw; q++) {
    if (type == 4 || type == 0) {
      sweep(A, type == 4 ? h->dinv[k] : h->djac[k], r, x, t);
      memcpy(x, t, sizeof(double) * (size_t)A->n);
    } else if (type == 1) {
      int fwd = (pass > 0) || (pass == 0 && q % 2 == 0);
      gs_pass(A, h->djac[k], r, x, fwd);
    } else {
      gs_pass(A, h->djac[k], r, x, 1);
      gs_pass(A, h->djac[k], r, x, 0);
    }
  }
}

static void smooth_zero(orc_h *h, int k, int type, int pass, const double *r, int nsw, double *x) {
  int32_t n = h->A[k].n;
  if (nsw <= 0) { for (int32_t i = 0; i < n; i++) x[i] = 0.0; return; }
  if (type == 4 || type == 0) {
    const double *d = (type == 4) ? h->dinv[k] : h->djac[k];
    ORC_ROWS
    for (int32_t i = 0; i < n; i++) x[i] = d[i] * r[i];
    smooth_more(h, k, type, pass, r, nsw - 1, x);
  } else {
    for (int32_t i = 0; i < n; i++) x[i] = 0.0;
    smooth_more(h, k, type, pass, r, nsw, x);
  }
}

/* Coarse-grid corrections per visit of level k (Appendix A cycle_type):
 * V-cycle 1; W-cycle 2 on every level; H-cycle (reading: the hybrid that
 * alternates them) 2 on odd levels and 1 on even ones.  With 2 the coarse
 * system is approximated by two cycles from zero: e = C(r_c), then
 * e += C(r_c - A_{k+1} e). */
static int corrections(const orc_h *h, int k) {
  if (h->p.cycle_type == 2) return 2;
  if (h->p.cycle_type == 1) return (k % 2 == 1) ? 2 : 1;
  return 1;
}

static void vcycle(orc_h *h, int k, const double *r, double *z) {
  const csr_t *A = &h->A[k];
  int32_t n = A->n;
  double *x = h->vx[k];
  if (k == h->nlev - 1) {
    if (h->coarse_dense) coarse_direct(h, r, z);
    else {
      smooth_zero(h, k, h->p.coarse_relax, 0, r, h->p.coarse_sweeps, x);
      memcpy(z, x, sizeof(double) * (size_t)n);
    }
    return;
  }
  smooth_zero(h, k, h->p.relax_type, 1, r, h->p.pre_sweeps, x);
  /* residual and restriction: r_c[I] = sum_{i in I, ascending} p_i (r - A x)_i */
  double *res = h->vres[k];
  spmv(A, x, res);
  ORC_ROWS
  for (int32_t i = 0; i < n; i++) res[i] = r[i] - res[i];
  int32_t nc = h->A[k + 1].n;
  double *rc = h->vr[k + 1];
  restrict_fold(n, nc, h->agg[k], h->pval[k], res, rc);
  double *ec = h->ve[k + 1];
  vcycle(h, k + 1, rc, ec);
  for (int g = 1; g < corrections(h, k); g++) {
    double *tc = h->vw[k + 1], *e2 = h->vz[k + 1];
    spmv(&h->A[k + 1], ec, tc);
    for (int32_t I = 0; I < nc; I++) tc[I] = rc[I] - tc[I];
    vcycle(h, k + 1, tc, e2);
    for (int32_t I = 0; I < nc; I++) ec[I] = ec[I] + e2[I];
  }
  ORC_ROWS
  for (int32_t i = 0; i < n; i++) x[i] = x[i] + h->pval[k][i] * ec[h->agg[k][i]];
  smooth_more(h, k, h->p.relax_type, -1, r, h->p.post_sweeps, x);
  memcpy(z, x, sizeof(double) * (size_t)n);
}

/* One hierarchy's preconditioner z = B r (binary64). */
static int single_apply(orc_h *h, const double *r, double *z) {
  if (!h->p.precond) { memcpy(z, r, sizeof(double) * (size_t)h->A[0].n); return ORC_OK; }
  vcycle(h, 0, r, z);
  return ORC_OK;
}

static int single_apply_f32(orc_h *h, const double *r, double *z);
static int composite_apply(orc_h *h, int m, int mixed, const double *r, double *z);

int orc_vcycle(orc_h *h, const double *r, double *z) {
  if (!h) return ORC_INVALID;
  return composite_apply(h, h->nhrc, 0, r, z);
}

/* ------------------------------------------------- binary32 V-cycle
 * Mixed-precision form: the same V-cycle evaluated in binary32.  Matrix
 * values and prolongator values are rounded to binary32; the l1 diagonal is
 * folded in binary32 from the rounded values.  The coarsest solve stays in
 * binary64 whichever solver it uses: its right-hand side is widened to
 * binary64, the direct solve (binary64 inverse) or the coarse_sweeps sweeps
 * (binary64 matrix and l1 diagonal) run as in the binary64 cycle, and the
 * result is rounded back.  Input and output stay binary64. */
static void spmv_f(const csr_t *A, const float *v, const float *x, float *y) {
  for (int32_t i = 0; i < A->n; i++) {
    float s = 0.0f;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) s = s + v[k] * x[A->ci[k]];
    y[i] = s;
  }
}

static void sweep_f(const csr_t *A, const float *v, const float *dinv, const float *r,
                    const float *x, float *xn) {
  for (int32_t i = 0; i < A->n; i++) {
    float s = 0.0f;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; k++) s = s + v[k] * x[A->ci[k]];
    xn[i] = x[i] + dinv[i] * (r[i] - s);
  }
}

static int build_f32(orc_h *h) {
  for (int k = 0; k < h->nlev; k++) {
    const csr_t *A = &h->A[k];
    size_t n = (size_t)A->n, z = (size_t)(A->nnz > 0 ? A->nnz : 1);
    h->fv[k] = (float *)malloc(sizeof(float) * z);
    h->fdinv[k] = (float *)malloc(sizeof(float) * n);
    h->fx[k] = (float *)malloc(sizeof(float) * n); h->ft[k] = (float *)malloc(sizeof(float) * n);
    h->fr[k] = (float *)malloc(sizeof(float) * n); h->fres[k] = (float *)malloc(sizeof(float) * n);
    h->fe[k] = (float *)malloc(sizeof(float) * n);
    if (!h->fv[k] || !h->fdinv[k] || !h->fx[k] || !h->ft[k] || !h->fr[k] || !h->fres[k] || !h->fe[k])
      return ORC_NOMEM;
    for (int64_t t = 0; t < A->nnz; t++) h->fv[k][t] = (float)A->v[t];
    for (int32_t i = 0; i < A->n; i++) {
      float m = 0.0f;
      for (int32_t t = A->rp[i]; t < A->rp[i + 1]; t++) m = m + fabsf(h->fv[k][t]);
      h->fdinv[k][i] = 1.0f / m;
    }
    if (k < h->nlev - 1) {
      h->fpval[k] = (float *)malloc(sizeof(float) * n);
      if (!h->fpval[k]) return ORC_NOMEM;
      for (int32_t i = 0; i < A->n; i++) h->fpval[k][i] = (float)h->pval[k][i];
    }
  }
  h->have_f32 = 1;
  return ORC_OK;
}

static void smooth_from_zero_f(const orc_h *h, int k, const float *r, int nsw, float *x, float *t) {
  const csr_t *A = &h->A[k];
  int32_t n = A->n;
  if (nsw <= 0) { for (int32_t i = 0; i < n; i++) x[i] = 0.0f; return; }
  for (int32_t i = 0; i < n; i++) x[i] = h->fdinv[k][i] * r[i];
  for (int s = 1; s < nsw; s++) {
    sweep_f(A, h->fv[k], h->fdinv[k], r, x, t);
    memcpy(x, t, sizeof(float) * (size_t)n);
  }
}

static void vcycle_f(orc_h *h, int k, const float *r, float *z) {
  const csr_t *A = &h->A[k];
  int32_t n = A->n;
  float *x = h->fx[k], *t = h->ft[k];
  if (k == h->nlev - 1) {
    double *rd = (double *)malloc(sizeof(double) * (size_t)n);
    double *zd = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; i++) rd[i] = (double)r[i];
    if (h->coarse_dense) coarse_direct(h, rd, zd);
    else smooth_from_zero(A, h->dinv[k], rd, h->p.coarse_sweeps, zd, h->vt[k]);
    for (int32_t i = 0; i < n; i++) z[i] = (float)zd[i];
    free(rd); free(zd);
    (void)x; (void)t;
    return;
  }
  smooth_from_zero_f(h, k, r, h->p.pre_sweeps, x, t);
  float *res = h->fres[k];
  spmv_f(A, h->fv[k], x, res);
  for (int32_t i = 0; i < n; i++) res[i] = r[i] - res[i];
  int32_t nc = h->A[k + 1].n;
  float *rc = h->fr[k + 1];
  for (int32_t I = 0; I < nc; I++) rc[I] = 0.0f;
  for (int32_t i = 0; i < n; i++) rc[h->agg[k][i]] = rc[h->agg[k][i]] + h->fpval[k][i] * res[i];
  float *ec = h->fe[k + 1];
  vcycle_f(h, k + 1, rc, ec);
  for (int32_t i = 0; i < n; i++) x[i] = x[i] + h->fpval[k][i] * ec[h->agg[k][i]];
  for (int s = 0; s < h->p.post_sweeps; s++) {
    sweep_f(A, h->fv[k], h->fdinv[k], r, x, t);
    memcpy(x, t, sizeof(float) * (size_t)n);
  }
  memcpy(z, x, sizeof(float) * (size_t)n);
}

/* z = B_32 r with r, z binary64 (single-level hierarchies use the binary64 solve). */
int orc_vcycle_f32(orc_h *h, const double *r, double *z) {
  if (!h) return ORC_INVALID;
  return composite_apply(h, h->nhrc, 1, r, z);
}

static int single_apply_f32(orc_h *h, const double *r, double *z) {
  int32_t n = h->A[0].n;
  if (!h->p.precond || h->nlev == 1) return single_apply(h, r, z);
  /* the binary32 cycle is the l1-Jacobi V-cycle */
  if (h->p.cycle_type != 0 || h->p.relax_type != 4 || h->p.coarse_relax != 4) return ORC_INVALID;
  if (!h->have_f32 && build_f32(h) != ORC_OK) return ORC_NOMEM;
  float *rf = (float *)malloc(sizeof(float) * (size_t)n);
  float *zf = (float *)malloc(sizeof(float) * (size_t)n);
  if (!rf || !zf) { free(rf); free(zf); return ORC_NOMEM; }
  for (int32_t i = 0; i < n; i++) rf[i] = (float)r[i];
  vcycle_f(h, 0, rf, zf);
  for (int32_t i = 0; i < n; i++) z[i] = (double)zf[i];
  free(rf); free(zf);
  return ORC_OK;
}

/* ------------------------------------------------- bootstrap composite
 * Appendix A lists a bootstrap AMG with up to max_hrc hierarchies combined by
 * a composition rule, built until the composite reaches a desired
 * convergence rate (the bootstrap of the cited BootCMatch papers).  With
 * B_1 .. B_m the hierarchies' preconditioners (each one V-cycle) and the
 * residual r:
 *   multiplicative (0):  z = B_1 r;  z += B_j (r - A z) for j = 2 .. m,
 *       so the error propagates by E = (I - B_m A) ... (I - B_1 A);
 *   symmetrized (1):     the same for j = 1 .. m, then for j = m-1 .. 1,
 *       E = (I - B_1 A) ... (I - B_m A) ... (I - B_1 A), an s.p.d. B;
 *   additive (2):        z = (B_1 r + ... + B_m r) / m (left fold, then the
 *       division): the average, so that the composite's stationary
 *       iteration converges whenever every B_j's does (a plain sum
 *       overcorrects by about a factor m; flexible CG itself is invariant
 *       under scaling B).
 * m = 1 is the plain preconditioner for every rule.  The outer product,
 * residuals and sums are binary64 also in the mixed-precision form (each
 * B_j is then the binary32 cycle). */
static int composite_apply(orc_h *h, int m, int mixed, const double *r, double *z) {
  orc_h *c0 = h;
  int32_t n = h->A[0].n;
  int st = mixed ? single_apply_f32(c0, r, z) : single_apply(c0, r, z);
  if (st != ORC_OK || m <= 1) return st;
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  double *e = (double *)malloc(sizeof(double) * (size_t)n);
  if (!t || !e) { free(t); free(e); return ORC_NOMEM; }
  int nsteps = (h->p.bootstrap_type == 1) ? 2 * m - 1 : m;
  for (int q = 1; q < nsteps && st == ORC_OK; q++) {
    int j = (q < m) ? q : 2 * m - 2 - q;       /* 0-based hierarchy of step q */
    orc_h *cj = (j == 0) ? h : h->hrc[j - 1];
    if (h->p.bootstrap_type == 2) {
      st = mixed ? single_apply_f32(cj, r, e) : single_apply(cj, r, e);
    } else {
      spmv(&h->A[0], z, t);
      for (int32_t i = 0; i < n; i++) t[i] = r[i] - t[i];
      st = mixed ? single_apply_f32(cj, t, e) : single_apply(cj, t, e);
    }
    for (int32_t i = 0; i < n; i++) z[i] = z[i] + e[i];
  }
  if (h->p.bootstrap_type == 2)
    for (int32_t i = 0; i < n; i++) z[i] = z[i] / (double)m;
  free(t); free(e);
  return st;
}

/* SplitMix64 (Steele, Lea and Flood 2014): the first output of a generator
 * whose state is c. */
static uint64_t splitmix64(uint64_t c) {
  uint64_t z = c + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Start vector of the rate estimate before hierarchy j + 1 is built:
 * x_i = 2 u - 1, u = (splitmix64(((16 seed + j) << 32) + i) >> 11) 2^-53. */
static void bootstrap_start(int32_t n, int32_t seed, int j, double *x) {
  uint64_t base = ((uint64_t)(uint32_t)(16 * seed + j)) << 32;
  for (int32_t i = 0; i < n; i++) {
    double u = (double)(splitmix64(base + (uint64_t)i) >> 11) * 0x1.0p-53;
    x[i] = 2.0 * u - 1.0;
  }
}

static double a_norm(const csr_t *A, const double *x, double *t) {
  spmv(A, x, t);
  return sqrt(dot(A->n, x, t));
}

/* Convergence-rate estimate of the composite of the first m hierarchies:
 * bootstrap_its steps of x <- x + B (0 - A x) on A x = 0 from the start
 * vector, rate = (||x_its||_A / ||x_0||_A)^(1 / its).  x holds x_its on
 * return. */
static int estimate_rate(orc_h *h, int m, double *x, double *rate) {
  const csr_t *A = &h->A[0];
  int32_t n = A->n;
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  double *e = (double *)malloc(sizeof(double) * (size_t)n);
  if (!t || !e) { free(t); free(e); return ORC_NOMEM; }
  bootstrap_start(n, h->p.bootstrap_seed, m, x);
  double n0 = a_norm(A, x, t);
  int st = ORC_OK;
  for (int it = 0; it < h->p.bootstrap_its && st == ORC_OK; it++) {
    spmv(A, x, t);
    for (int32_t i = 0; i < n; i++) t[i] = 0.0 - t[i];
    st = composite_apply(h, m, 0, t, e);
    for (int32_t i = 0; i < n; i++) x[i] = x[i] + e[i];
  }
  double nf = a_norm(A, x, t);
  *rate = pow(nf / n0, 1.0 / (double)h->p.bootstrap_its);
  free(t); free(e);
  return st;
}

/* Bootstrap setup: hierarchy 1 from the configured smooth vector; then, while
 * fewer than max_hrc hierarchies exist and the composite's estimated rate is
 * above bootstrap_rate, the estimate's final iterate (the error the
 * composite reduces slowest), scaled by its largest magnitude, is the smooth
 * vector of a new hierarchy with the same parameters.  The rate of the final
 * composite is estimated as well (rate[nhrc - 1]). */
orc_h *orc_setup(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                 const orc_params *par, const double *w_given, int *status) {
  orc_h *h = build_single(n, rp, ci, v, par, w_given, status);
  if (!h) return NULL;
  h->nhrc = 1;
  if (par->max_hrc <= 1 || !par->precond) return h;
  double *x = (double *)malloc(sizeof(double) * (size_t)n);
  if (!x) { orc_free(h); *status = ORC_NOMEM; return NULL; }
  orc_params pc = *par;
  pc.max_hrc = 1;
  pc.smooth_vec = 2;
  for (;;) {
    double rate;
    *status = estimate_rate(h, h->nhrc, x, &rate);
    if (*status != ORC_OK) break;
    h->rate[h->nrate++] = rate;
    if (rate <= par->bootstrap_rate || h->nhrc >= par->max_hrc) break;
    double mx = 0.0;
    int finite = 1;
    for (int32_t i = 0; i < n; i++) {
      if (!isfinite(x[i])) finite = 0;
      else if (fabs(x[i]) > mx) mx = fabs(x[i]);
    }
    if (!finite || !(mx > 0.0)) break;
    for (int32_t i = 0; i < n; i++) x[i] = x[i] / mx;
    orc_h *c = build_single(n, rp, ci, v, &pc, x, status);
    if (!c) break;
    c->nhrc = 1;
    h->hrc[h->nhrc - 1] = c;
    h->nhrc++;
  }
  free(x);
  if (*status != ORC_OK) { orc_free(h); return NULL; }
  return h;
}

int orc_nhrc(const orc_h *h) { return h ? h->nhrc : 0; }

/* The preconditioner of hierarchy h alone (its V-cycle), also when h heads a
 * composite. */
int orc_vcycle_single(orc_h *h, const double *r, double *z) {
  if (!h) return ORC_INVALID;
  return single_apply(h, r, z);
}

/* Rate estimates: out[j-1] = estimated rate of the composite of the first j
 * hierarchies; returns how many were taken. */
int orc_rates(const orc_h *h, double *out) {
  if (!h) return 0;
  for (int j = 0; j < h->nrate; j++) out[j] = h->rate[j];
  return h->nrate;
}

/* Hierarchy j (0-based) of the composite, owned by h. */
orc_h *orc_component(orc_h *h, int j) {
  if (!h || j < 0 || j >= h->nhrc) return NULL;
  return j == 0 ? h : h->hrc[j - 1];
}

/* ------------------------------------------------------------- flexible CG
 * Alg. 1 (Notay's flexible PCG, Sec. 3).  u holds u_0 on entry, the solution on exit.
 * Stop when ||r_i||_2 <= rtol ||r_0||_2 (recurrence residual, tested after
 * every update of r) or after maxit preconditioner applications (Sec. 5); the
 * iteration count is the number of applications of B.  rho <= 0 (or not
 * finite) means A or B is not s.p.d. */
static int pcg_impl(orc_h *h, const double *b, double *u, double rtol, int32_t maxit,
                    int32_t *iters, double *relres, int mixed) {
  if (!h || !b || !u || !(rtol > 0.0) || maxit < 1) return ORC_INVALID;
  const csr_t *A = &h->A[0];
  int32_t n = A->n;
  for (int32_t i = 0; i < n; i++) if (!isfinite(b[i]) || !isfinite(u[i])) return ORC_NONFINITE;
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  double *v = (double *)malloc(sizeof(double) * (size_t)n);
  double *d = (double *)malloc(sizeof(double) * (size_t)n);
  double *q = (double *)malloc(sizeof(double) * (size_t)n);
  if (!r || !w || !v || !d || !q) { free(r); free(w); free(v); free(d); free(q); return ORC_NOMEM; }
  int status = ORC_OK;
  spmv(A, u, r);
  for (int32_t i = 0; i < n; i++) r[i] = b[i] - r[i];
  double nr0 = sqrt(dot(n, r, r));
  int32_t it = 0;
  double rel = 0.0;
  if (nr0 == 0.0) goto done;

  /* initial step */
  if (mixed) orc_vcycle_f32(h, r, w); else orc_vcycle(h, r, w);
  it = 1;
  spmv(A, w, v);
  double alpha = dot(n, w, r);
  double beta = dot(n, w, v);
  double rho = beta;
  if (!isfinite(rho) || !isfinite(alpha)) { status = ORC_NONFINITE; goto done; }
  if (!(rho > 0.0)) { status = ORC_NOT_SPD; goto done; }
  memcpy(d, w, sizeof(double) * (size_t)n);
  memcpy(q, v, sizeof(double) * (size_t)n);
  double a = alpha / rho;
  for (int32_t i = 0; i < n; i++) u[i] = u[i] + a * d[i];
  for (int32_t i = 0; i < n; i++) r[i] = r[i] - a * q[i];
  double nr = sqrt(dot(n, r, r));
  rel = nr / nr0;
  while (!(nr <= rtol * nr0)) {
    if (!isfinite(nr)) { status = ORC_NONFINITE; goto done; }
    if (it >= maxit) { status = ORC_NOT_CONVERGED; goto done; }
    if (mixed) orc_vcycle_f32(h, r, w); else orc_vcycle(h, r, w);
    it++;
    spmv(A, w, v);
    alpha = dot(n, w, r);
    beta = dot(n, w, v);
    double gamma = dot(n, w, q);
    double rho_new = beta - (gamma * gamma) / rho;
    if (!isfinite(rho_new) || !isfinite(alpha)) { status = ORC_NONFINITE; goto done; }
    if (!(rho_new > 0.0)) { status = ORC_NOT_SPD; goto done; }
    double c = gamma / rho;
    a = alpha / rho_new;
    ORC_ROWS
    for (int32_t i = 0; i < n; i++) {
      d[i] = w[i] - c * d[i];
      u[i] = u[i] + a * d[i];
      q[i] = v[i] - c * q[i];
      r[i] = r[i] - a * q[i];
    }
    rho = rho_new;
    nr = sqrt(dot(n, r, r));
    rel = nr / nr0;
  }
done:
  *iters = it;
  *relres = rel;
  free(r); free(w); free(v); free(d); free(q);
  return status;
}

int orc_pcg(orc_h *h, const double *b, double *u, double rtol, int32_t maxit,
            int32_t *iters, double *relres) {
  return pcg_impl(h, b, u, rtol, maxit, iters, relres, 0);
}

/* Flexible CG with the binary32 V-cycle (mixed-precision form). */
int orc_pcg_mixed(orc_h *h, const double *b, double *u, double rtol, int32_t maxit,
                  int32_t *iters, double *relres) {
  return pcg_impl(h, b, u, rtol, maxit, iters, relres, 1);
}

/* ------------------------------------------------------------ introspection */

int orc_nlevels(const orc_h *h) { return h ? h->nlev : 0; }
int orc_coarse_dense(const orc_h *h) { return h ? h->coarse_dense : 0; }

int orc_level_size(const orc_h *h, int k, int32_t *n, int64_t *nnz) {
  if (!h || k < 0 || k >= h->nlev) return ORC_INVALID;
  *n = h->A[k].n; *nnz = h->A[k].nnz;
  return ORC_OK;
}

/* OPC = sum_k nnz(A^k) / nnz(A^0)  (Sec. 5). */
double orc_opc(const orc_h *h) {
  double s = 0.0;
  for (int k = 0; k < h->nlev; k++) s += (double)h->A[k].nnz;
  return s / (double)h->A[0].nnz;
}

/* Copy level k out: CSR arrays (sized by orc_level_size), the smooth vector,
 * and for k < nlev-1 the aggregate map and P values.  NULL pointers skip. */
int orc_export_level(const orc_h *h, int k, int32_t *rp, int32_t *ci, double *v,
                     double *w, int32_t *agg, double *pval, double *dinv) {
  if (!h || k < 0 || k >= h->nlev) return ORC_INVALID;
  const csr_t *A = &h->A[k];
  if (rp) memcpy(rp, A->rp, sizeof(int32_t) * (size_t)(A->n + 1));
  if (ci) memcpy(ci, A->ci, sizeof(int32_t) * (size_t)A->nnz);
  if (v) memcpy(v, A->v, sizeof(double) * (size_t)A->nnz);
  if (w) memcpy(w, h->w[k], sizeof(double) * (size_t)A->n);
  if (dinv) memcpy(dinv, h->dinv[k], sizeof(double) * (size_t)A->n);
  if (k < h->nlev - 1) {
    if (agg) memcpy(agg, h->agg[k], sizeof(int32_t) * (size_t)A->n);
    if (pval) memcpy(pval, h->pval[k], sizeof(double) * (size_t)A->n);
  }
  return ORC_OK;
}

/* Inverse of the coarsest matrix (n_c x n_c, row-major). */
int orc_export_coarse_inverse(const orc_h *h, double *Ainv) {
  if (!h || !h->coarse_dense) return ORC_INVALID;
  int32_t m = h->A[h->nlev - 1].n;
  memcpy(Ainv, h->Ainv, sizeof(double) * (size_t)m * m);
  return ORC_OK;
}

/* Dense Cholesky factor of the coarsest level (n_c x n_c, row-major). */
int orc_export_coarse_factor(const orc_h *h, double *L) {
  if (!h || !h->coarse_dense) return ORC_INVALID;
  int32_t m = h->A[h->nlev - 1].n;
  memcpy(L, h->L, sizeof(double) * (size_t)m * m);
  return ORC_OK;
}

/* One pairwise coarsening step on a given matrix, for tests: matching,
 * aggregates, P values, coarse vector and coarse matrix (caller frees via
 * orc_free_csr_arrays). */
int orc_pairwise_step(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                      const double *w, const int32_t *part, int32_t *mate, int32_t *agg,
                      double *pval, int32_t *nc_out, double **wc_out, int32_t **crp,
                      int32_t **cci, double **cv, int64_t *cnnz) {
  csr_t A = {n, rp[n], (int32_t *)rp, (int32_t *)ci, (double *)v};
  int st = match_greedy(&A, w, part, mate);
  if (st != ORC_OK) return st;
  int32_t nc = aggregate_ids(n, mate, agg);
  pair_pvals(n, mate, w, pval);
  double *wc = (double *)malloc(sizeof(double) * (size_t)nc);
  csr_t Ac;
  if (!wc) return ORC_NOMEM;
  st = galerkin(&A, nc, agg, pval, &Ac);
  if (st != ORC_OK) { free(wc); return st; }
  restrict_fold(n, nc, agg, pval, w, wc);
  *nc_out = nc; *wc_out = wc; *crp = Ac.rp; *cci = Ac.ci; *cv = Ac.v; *cnnz = Ac.nnz;
  return ORC_OK;
}

/* Row block of every row of level k (decoupled aggregation). */
int orc_export_part(const orc_h *h, int k, int32_t *part) {
  if (!h || k < 0 || k >= h->nlev) return ORC_INVALID;
  memcpy(part, h->part[k], sizeof(int32_t) * (size_t)h->A[k].n);
  return ORC_OK;
}

void orc_free_ptr(void *p) { free(p); }
