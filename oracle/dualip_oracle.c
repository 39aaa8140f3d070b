/*
 * FP64 CPU oracle for ridge-regularized matching-LP dual ascent.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path: it is a plain, slow, obviously-correct restatement of the
 * paper's method so that the GPU results can be checked against it.
 *
 * What it computes, following the paper:
 *   primal (eq. 1)     min_{x in C} c^T x + (gamma/2)||x||^2  s.t.  A x <= b
 *   dual (eq. 2)       g(lam) = min_{x in C} c^T x + (gamma/2)||x||^2 + lam^T (A x - b)
 *   recovery (eq. 3)   x*(lam) = Pi_C( -(A^T lam + c) / gamma )
 *   gradient (eq. 4)   grad g(lam) = A x*(lam) - b      (Danskin)
 *   A                  Definition 1: m families, each a horizontal stack of
 *                      diagonal per-user blocks, stored as user-major CSR
 *   Pi_C               per-user simplex {x >= 0, sum x <= z} (or = z), or box
 *                      [0,u] (Section 3.3); simplex by the sort-based method of
 *                      Duchi et al. (Section 4.3)
 *   Jacobi scaling     D = diag(1/||A_r||_2), 1 on zero rows; A' = DA, b' = Db
 *                      (Appendix C, "Jacobi preconditioning")
 *   step               eta = gamma / Lhat with Lhat >= ||A'||_2^2, since the
 *                      gradient's Lipschitz constant is at most ||A||^2/gamma
 *                      and the step follows gamma (Appendix C, "Regularization
 *                      decay")
 *   ascent             accelerated projected gradient on lam >= 0 with a
 *                      momentum vector (Section 4.4); FISTA form
 *   continuation       gamma decreases stage by stage, each stage warm-started
 *                      from the previous dual iterate (Section 6)
 *
 * Readings where the paper is silent are listed in the design notes; the ones
 * coded here: FISTA momentum with reset at every stage switch; the simplex
 * early exit tests sum(max(v,0)) <= z exactly; the duality gap is certified
 * with a feasible repair of x*(lam) (item-wise scaling by min(1, b/Ax)).
 *
 * Reductions over users run in a fixed number of chunks merged in chunk
 * order, so results do not depend on the OpenMP thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_SIMPLEX_LE = 0, ORC_SIMPLEX_EQ = 1, ORC_BOX = 2, ORC_BOXCUT = 3 };

typedef struct {
  int64_t n_users;
  int32_t n_items;
  int32_t n_families;
  const int64_t* row_ptr; /* I+1 */
  const int32_t* item_idx; /* nnz */
  const float* c;          /* nnz */
  const float* a;          /* m*nnz family-major, or NULL: every a_kij = 1 */
  const double* b;         /* m*J */
  int32_t proj;
  int32_t eq_mask;         /* bit k: family k holds equality rows A_k x = b_k (free duals) */
  double radius;           /* z: simplex sum / box bound / box-cut sum */
  double upper;            /* u of the box-cut set {0 <= x <= u, sum x <= z} */
  int32_t global_count;    /* 1: one more coupling row, sum over all (i,j) of x_ij <= global_cap */
  double global_cap;       /* M of the global-count row */
} orc_inst;

/*
 * Dual coordinates: the m*J item rows (family-major), then, with a global-count
 * row (Section 5: one more coupling constraint sum_{(i,j) in E} x_ij <= M, i.e.
 * one more row of A whose coefficients are all 1), one more coordinate at
 * index m*J.
 */
static inline int64_t n_rows(const orc_inst* P) {
  return (int64_t)P->n_families * P->n_items + (P->global_count ? 1 : 0);
}
static inline double row_b(const orc_inst* P, int64_t r) {
  const int64_t mJ = (int64_t)P->n_families * P->n_items;
  return r < mJ ? P->b[r] : P->global_cap;
}

#define ORC_CHUNKS 64

static inline double coef(const orc_inst* P, int k, int64_t e) {
  int64_t nnz = P->row_ptr[P->n_users];
  return P->a ? (double)P->a[(int64_t)k * nnz + e] : 1.0;
}

/* ------------------------------------------------------------------------ */
/* Projections                                                               */
/* ------------------------------------------------------------------------ */
static int cmp_desc(const void* p, const void* q) {
  double x = *(const double*)p, y = *(const double*)q;
  return (x < y) - (x > y);
}

/*
 * Euclidean projection of v (length d) onto {x >= 0, sum x <= z} (eq = 0)
 * or {x >= 0, sum x = z} (eq = 1).  Duchi et al. 2008: sort descending,
 * rho = max{ r : u_r - (sum_{q<=r} u_q - z)/r > 0 }, theta = (sum_{q<=rho} u_q - z)/rho,
 * x = max(v - theta, 0).  For the inequality set, a point whose positive part
 * already sums to at most z is projected by clamping at zero.
 */
void orc_project_simplex(const double* v, int64_t d, double z, int eq, double* x) {
  if (d <= 0) return;
  if (!eq) {
    double spos = 0.0;
    for (int64_t e = 0; e < d; ++e) spos += v[e] > 0.0 ? v[e] : 0.0;
    if (spos <= z) {
      for (int64_t e = 0; e < d; ++e) x[e] = v[e] > 0.0 ? v[e] : 0.0;
      return;
    }
  }
  double* u = (double*)malloc(sizeof(double) * (size_t)d);
  memcpy(u, v, sizeof(double) * (size_t)d);
  qsort(u, (size_t)d, sizeof(double), cmp_desc);
  double cum = 0.0, theta = 0.0;
  for (int64_t r = 1; r <= d; ++r) {
    cum += u[r - 1];
    double t = (cum - z) / (double)r;
    if (u[r - 1] - t > 0.0) theta = t;
  }
  for (int64_t e = 0; e < d; ++e) {
    double y = v[e] - theta;
    x[e] = y > 0.0 ? y : 0.0;
  }
  free(u);
}

/* Projection onto the box [0, u]^d. */
void orc_project_box(const double* v, int64_t d, double u, double* x) {
  for (int64_t e = 0; e < d; ++e) x[e] = v[e] < 0.0 ? 0.0 : (v[e] > u ? u : v[e]);
}

static int cmp_asc(const void* p, const void* q) {
  double x = *(const double*)p, y = *(const double*)q;
  return (x > y) - (x < y);
}

static double boxcut_sum(const double* v, int64_t d, double u, double theta) {
  double f = 0.0;
  for (int64_t e = 0; e < d; ++e) {
    double y = v[e] - theta;
    f += y < 0.0 ? 0.0 : (y > u ? u : y);
  }
  return f;
}

/*
 * Euclidean projection onto the box-cut set {0 <= x <= u, sum x <= z} (the
 * ProjectionMap primitive named in Table 1).  KKT: x = clamp(v - theta, 0, u)
 * with theta = 0 if clamp(v, 0, u) sums to at most z, else theta > 0 with
 * f(theta) = sum clamp(v - theta, 0, u) = z.  f is continuous, nonincreasing
 * and linear between the breakpoints {v_e, v_e - u}; bisection over the sorted
 * breakpoints finds the piece where f crosses z, and on that piece the free
 * coordinates F and capped coordinates C give theta = (|C| u + sum_F v - z) / |F|.
 */
void orc_project_boxcut(const double* v, int64_t d, double u, double z, double* x) {
  if (d <= 0) return;
  if (boxcut_sum(v, d, u, 0.0) <= z) {
    for (int64_t e = 0; e < d; ++e) x[e] = v[e] < 0.0 ? 0.0 : (v[e] > u ? u : v[e]);
    return;
  }
  double* bp = (double*)malloc(sizeof(double) * (size_t)(2 * d + 1));
  int64_t n = 0;
  bp[n++] = 0.0;
  for (int64_t e = 0; e < d; ++e) {
    if (v[e] > 0.0) bp[n++] = v[e];
    if (v[e] - u > 0.0) bp[n++] = v[e] - u;
  }
  qsort(bp, (size_t)n, sizeof(double), cmp_asc);
  /* f(bp[0] = 0) > z and f(bp[n-1] = max v) = 0 <= z: find lo < hi adjacent with f(lo) > z >= f(hi) */
  int64_t lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) / 2;
    if (boxcut_sum(v, d, u, bp[mid]) > z) lo = mid;
    else hi = mid;
  }
  double theta;
  if (bp[hi] <= bp[lo]) {
    theta = bp[hi];
  } else {
    const double tm = 0.5 * (bp[lo] + bp[hi]);
    double cnt = 0.0, sfree = 0.0, capped = 0.0;
    for (int64_t e = 0; e < d; ++e) {
      double y = v[e] - tm;
      if (y >= u) capped += u;
      else if (y > 0.0) { cnt += 1.0; sfree += v[e]; }
    }
    theta = cnt > 0.0 ? (capped + sfree - z) / cnt : bp[hi];
  }
  free(bp);
  for (int64_t e = 0; e < d; ++e) {
    double y = v[e] - theta;
    x[e] = y < 0.0 ? 0.0 : (y > u ? u : y);
  }
}

static void project_row(const orc_inst* P, const double* v, int64_t d, double* x) {
  if (P->proj == ORC_BOX) orc_project_box(v, d, P->radius, x);
  else if (P->proj == ORC_BOXCUT) orc_project_boxcut(v, d, P->upper, P->radius, x);
  else orc_project_simplex(v, d, P->radius, P->proj == ORC_SIMPLEX_EQ, x);
}

/* ProjectionMap: x = Pi_C(v) row by row, v and x of length nnz. */
int orc_project_rows(const orc_inst* P, const double* v, double* x) {
  const int64_t I = P->n_users;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < I; ++i) {
    int64_t s = P->row_ptr[i], d = P->row_ptr[i + 1] - s;
    project_row(P, v + s, d, x + s);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* ObjectiveFunction.calculate (Table 1): g(lam), grad g(lam), x*(lam)        */
/* ------------------------------------------------------------------------ */
/*
 * lam (m*J) in the problem's own units.  Outputs:
 *   ax[m*J]     A x*(lam)                      (nullable)
 *   grad[m*J]   A x*(lam) - b                  (nullable)
 *   gval        g(lam)                         (nullable)
 *   x[nnz]      x*(lam)                        (nullable)
 *   cx, xx      c^T x*, ||x*||^2               (nullable)
 */
int orc_dual_grad_ex(const orc_inst* P, const double* lam, double gamma, double* ax_out,
                     double* grad, double* gval, double* x_out, double* cx_out, double* xx_out) {
  if (!(gamma > 0.0)) return -1;
  const int64_t I = P->n_users;
  const int32_t J = P->n_items, m = P->n_families;
  const int64_t mJ = (int64_t)m * J, nr = n_rows(P);
  const double lam_g = P->global_count ? lam[mJ] : 0.0;  /* the global row's dual */
  double* part = (double*)calloc((size_t)ORC_CHUNKS * (size_t)(nr + 3), sizeof(double));
  if (!part) return -2;

#pragma omp parallel for schedule(dynamic, 1)
  for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
    double* acc = part + (size_t)ch * (size_t)(nr + 3);
    int64_t u0 = I * ch / ORC_CHUNKS, u1 = I * (ch + 1) / ORC_CHUNKS;
    int64_t cap = 0;
    double *v = NULL, *x = NULL, *s = NULL;
    for (int64_t i = u0; i < u1; ++i) {
      int64_t r0 = P->row_ptr[i], d = P->row_ptr[i + 1] - r0;
      if (d > cap) {
        cap = d;
        v = (double*)realloc(v, sizeof(double) * (size_t)cap);
        x = (double*)realloc(x, sizeof(double) * (size_t)cap);
        s = (double*)realloc(s, sizeof(double) * (size_t)cap);
      }
      for (int64_t e = 0; e < d; ++e) {
        int32_t j = P->item_idx[r0 + e];
        double sum = 0.0;
        for (int k = 0; k < m; ++k) sum += coef(P, k, r0 + e) * lam[(int64_t)k * J + j];
        sum += lam_g;                                       /* the global row's coefficient is 1 */
        s[e] = sum;                                         /* (A^T lam)_ij */
        v[e] = -((double)P->c[r0 + e] + sum) / gamma;       /* eq. 3 argument */
      }
      project_row(P, v, d, x);
      for (int64_t e = 0; e < d; ++e) {
        int32_t j = P->item_idx[r0 + e];
        double cij = (double)P->c[r0 + e];
        for (int k = 0; k < m; ++k) acc[(int64_t)k * J + j] += coef(P, k, r0 + e) * x[e];
        if (P->global_count) acc[mJ] += x[e];
        acc[nr] += cij * x[e];
        acc[nr + 1] += x[e] * x[e];
        acc[nr + 2] += s[e] * x[e];
        if (x_out) x_out[r0 + e] = x[e];
      }
    }
    free(v); free(x); free(s);
  }
  double* ax = (double*)calloc((size_t)nr, sizeof(double));
  double cx = 0.0, xx = 0.0, sx = 0.0;
  for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
    const double* acc = part + (size_t)ch * (size_t)(nr + 3);
    for (int64_t r = 0; r < nr; ++r) ax[r] += acc[r];
    cx += acc[nr];
    xx += acc[nr + 1];
    sx += acc[nr + 2];
  }
  double lb = 0.0;
  for (int64_t r = 0; r < nr; ++r) lb += lam[r] * row_b(P, r);
  if (ax_out) memcpy(ax_out, ax, sizeof(double) * (size_t)nr);
  if (grad) for (int64_t r = 0; r < nr; ++r) grad[r] = ax[r] - row_b(P, r);
  /* eq. 2 at its minimiser: c^T x + (gamma/2)||x||^2 + lam^T A x - lam^T b */
  if (gval) *gval = cx + 0.5 * gamma * xx + sx - lb;
  if (cx_out) *cx_out = cx;
  if (xx_out) *xx_out = xx;
  free(ax);
  free(part);
  return 0;
}

int orc_dual_grad(const orc_inst* P, const double* lam, double gamma, double* grad, double* gval,
                  double* x_out) {
  return orc_dual_grad_ex(P, lam, gamma, NULL, grad, gval, x_out, NULL, NULL);
}

/* Primal objective c^T x + (gamma/2)||x||^2 and A x for a given x (nnz). */
int orc_primal(const orc_inst* P, const double* x, double gamma, double* pobj, double* ax_out) {
  const int64_t nnz = P->row_ptr[P->n_users];
  const int32_t J = P->n_items, m = P->n_families;
  const int64_t mJ = (int64_t)m * J;
  double cx = 0.0, xx = 0.0;
  if (ax_out) memset(ax_out, 0, sizeof(double) * (size_t)n_rows(P));
  for (int64_t e = 0; e < nnz; ++e) {
    cx += (double)P->c[e] * x[e];
    xx += x[e] * x[e];
    if (ax_out) {
      for (int k = 0; k < m; ++k) ax_out[(int64_t)k * J + P->item_idx[e]] += coef(P, k, e) * x[e];
      if (P->global_count) ax_out[mJ] += x[e];
    }
  }
  if (pobj) *pobj = cx + 0.5 * gamma * xx;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Jacobi scaling and the step bound                                         */
/* ------------------------------------------------------------------------ */
/*
 * D[k*J+j] = 1/||A_{kj}||_2 (1 on zero rows) when jacobi, else 1.
 * Lhat >= lambda_max(A' A'^T) with A' = D A.  A'A'^T is block diagonal over
 * items with m x m blocks M_j[k][l] = sum_i a'_kij a'_lij (Definition 1: a row
 * of family k at item j only meets columns (i, j)).  For m = 1 the blocks are
 * scalars and Lhat is exact; for m > 1 it is the Gershgorin row-sum bound.
 */
int orc_scaling(const orc_inst* P, int jacobi, double* D, double* Lhat) {
  const int64_t nnz = P->row_ptr[P->n_users];
  const int32_t J = P->n_items, m = P->n_families;
  const int64_t mJ = (int64_t)m * J;
  double* M = (double*)calloc((size_t)J * (size_t)m * (size_t)m, sizeof(double));
  for (int64_t e = 0; e < nnz; ++e) {
    int32_t j = P->item_idx[e];
    for (int k = 0; k < m; ++k)
      for (int l = 0; l < m; ++l) M[((int64_t)j * m + k) * m + l] += coef(P, k, e) * coef(P, l, e);
  }
  for (int64_t r = 0; r < mJ; ++r) D[r] = 1.0;
  if (jacobi) {
    for (int k = 0; k < m; ++k)
      for (int32_t j = 0; j < J; ++j) {
        double nrm2 = M[((int64_t)j * m + k) * m + k];
        D[(int64_t)k * J + j] = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 1.0;
      }
  }
  double L = 0.0;
  for (int32_t j = 0; j < J; ++j)
    for (int k = 0; k < m; ++k) {
      double row = 0.0;
      for (int l = 0; l < m; ++l)
        row += fabs(D[(int64_t)k * J + j] * M[((int64_t)j * m + k) * m + l] * D[(int64_t)l * J + j]);
      if (row > L) L = row;
    }
  if (P->global_count) {
    /* The global row g (all ones, scaled by D_g = 1/sqrt(nnz)) adds one row and
     * column to A'A'^T: diagonal d_g = D_g^2 nnz and couplings c_kj = D_kj D_g
     * sum_i a_kij.  Splitting A'A'^T into its block diagonal (the item blocks and
     * d_g) plus the off-diagonal part [[0, c], [c^T, 0]], whose largest eigenvalue
     * is ||c||_2, Weyl's inequality bounds lambda_max by max(L_items, d_g) + ||c||_2. */
    const double Dg = (jacobi && nnz > 0) ? 1.0 / sqrt((double)nnz) : 1.0;
    D[mJ] = Dg;
    double* colsum = (double*)calloc((size_t)mJ, sizeof(double));
    for (int64_t e = 0; e < nnz; ++e)
      for (int k = 0; k < m; ++k) colsum[(int64_t)k * J + P->item_idx[e]] += coef(P, k, e);
    double c2 = 0.0;
    for (int64_t r = 0; r < mJ; ++r) {
      const double c = D[r] * Dg * colsum[r];
      c2 += c * c;
    }
    const double dg = Dg * Dg * (double)nnz;
    L = (L > dg ? L : dg) + sqrt(c2);
    free(colsum);
  }
  *Lhat = L;
  free(M);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Certificate: feasible repair, primal value, gap, slack                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t iters;
  double gamma;
  double dual_obj;   /* g_gamma(lam) */
  double primal_obj; /* P_gamma(x~) of the repaired primal */
  double rel_gap;    /* (P_gamma(x~) - g_gamma(lam)) / max(1, |g_gamma(lam)|) */
  double max_slack;  /* max_r (A x*(lam) - b)_r^+ */
  double lagr_gap;   /* -lam^T grad g(lam) = P_gamma(x*) - g_gamma(lam) */
  int32_t status;    /* 0 converged, 1 not converged, -1 error */
  int32_t stage;
} orc_stats;

/*
 * At lam: x = x*(lam); r_j = min_k min(1, b_kj / (A_k x)_j) (1 when (A_k x)_j
 * <= b_kj); x~_ij = r_j x_ij is feasible when a >= 0, b >= 0 and C is closed
 * under scaling toward 0 (simplex-LE, box, box-cut).  Weak duality gives
 * g(lam) <= P(x~).  Equality rows have no such repair: with any of them the
 * gap is NaN and the slack is max |A x - b| over them.
 */
int orc_certificate(const orc_inst* P, const double* lam, double gamma, orc_stats* st) {
  const int64_t nnz = P->row_ptr[P->n_users];
  const int32_t J = P->n_items, m = P->n_families;
  const int64_t mJ = (int64_t)m * J;
  double* x = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  double* ax = (double*)malloc(sizeof(double) * (size_t)n_rows(P));
  double gval = 0.0, cx = 0.0, xx = 0.0;
  orc_dual_grad_ex(P, lam, gamma, ax, NULL, &gval, x, &cx, &xx);
  double* r = (double*)malloc(sizeof(double) * (size_t)J);
  double slack = 0.0, lg = 0.0;
  /* global-count row: scaling every x by rho = min(1, M / sum x) makes it
   * feasible and keeps every item row feasible (their factors only shrink) */
  double rho = 1.0;
  if (P->global_count) {
    const double G = ax[mJ], M = P->global_cap, viol = G - M;
    if (viol > slack) slack = viol;
    lg -= lam[mJ] * viol;
    if (G > M) rho = M > 0.0 ? M / G : 0.0;
  }
  for (int32_t j = 0; j < J; ++j) r[j] = rho;
  for (int k = 0; k < m; ++k)
    for (int32_t j = 0; j < J; ++j) {
      int64_t q = (int64_t)k * J + j;
      double viol = ax[q] - P->b[q];
      const int eq = (P->eq_mask >> k) & 1;
      if ((eq ? fabs(viol) : viol) > slack) slack = eq ? fabs(viol) : viol;
      lg -= lam[q] * viol;
      if (!eq && ax[q] > P->b[q]) {
        double f = P->b[q] > 0.0 ? P->b[q] / ax[q] : 0.0;
        if (f < r[j]) r[j] = f;
      }
    }
  double pc = 0.0, pq = 0.0;
  for (int64_t e = 0; e < nnz; ++e) {
    double xt = r[P->item_idx[e]] * x[e];
    pc += (double)P->c[e] * xt;
    pq += xt * xt;
  }
  double pobj = pc + 0.5 * gamma * pq;
  st->gamma = gamma;
  st->dual_obj = gval;
  st->primal_obj = pobj;
  st->rel_gap = (P->eq_mask & ((1 << m) - 1)) ? NAN : (pobj - gval) / fmax(1.0, fabs(gval));
  st->max_slack = slack;
  st->lagr_gap = lg;
  free(x); free(ax); free(r);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Maximizer: accelerated projected dual ascent with continuation            */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_stages;
  int32_t jacobi;
  const double* gammas;   /* n_stages */
  const int64_t* iters;   /* n_stages; -1 on the last stage = until tol */
  double tol;             /* relative certified gap */
  int64_t max_iters;      /* total cap */
  int32_t check_every;    /* certificate period in the final stage */
  int32_t reset_momentum; /* reset t and y at stage switches */
  double step_scale;      /* eta = step_scale * gamma / Lhat */
  int64_t n_snap;         /* trajectory snapshots of lam (problem units) */
  const int64_t* snap_iters;
  double* snap_lambda;    /* n_snap * m*J */
  double* trace_dual;     /* nullable, g(lam_t) for t = 1..max_iters (expensive) */
} orc_solve_opts;

int orc_solve(const orc_inst* P, const orc_solve_opts* o, const double* lam0, double* lam_out,
              orc_stats* st) {
  const int32_t J = P->n_items;
  const int64_t mJ = n_rows(P);  /* dual coordinates: item rows, then the global-count row */
  if (o->n_stages <= 0) return -1;
  double* D = (double*)malloc(sizeof(double) * (size_t)mJ);
  double Lhat = 0.0;
  orc_scaling(P, o->jacobi, D, &Lhat);
  if (!(Lhat > 0.0)) Lhat = 1.0;
  /* scaled dual lam' with lam = D lam' (the dual of A'x <= b') */
  double* lp = (double*)malloc(sizeof(double) * (size_t)mJ);  /* lam'_t */
  double* yp = (double*)malloc(sizeof(double) * (size_t)mJ);  /* y'_t   */
  double* yo = (double*)malloc(sizeof(double) * (size_t)mJ);  /* D y'   */
  double* gr = (double*)malloc(sizeof(double) * (size_t)mJ);
  double* lo = (double*)malloc(sizeof(double) * (size_t)mJ);
  for (int64_t r = 0; r < mJ; ++r) {
    const int eq = (P->eq_mask >> (int)(r / J)) & 1;
    double l = lam0 ? lam0[r] / D[r] : 0.0;
    lp[r] = (eq || l > 0.0) ? l : 0.0;
    yp[r] = lp[r];
  }
  int64_t it = 0, snap = 0;
  orc_stats cs;
  memset(&cs, 0, sizeof(cs));
  cs.status = 1;
  int done = 0;
  for (int32_t s = 0; s < o->n_stages && !done; ++s) {
    const double gamma = o->gammas[s];
    const double eta = o->step_scale * gamma / Lhat;
    const int last = (s == o->n_stages - 1);
    const int64_t n_it = o->iters[s];
    double tk = 1.0;
    if (o->reset_momentum) memcpy(yp, lp, sizeof(double) * (size_t)mJ);
    for (int64_t k = 0; (n_it < 0 || k < n_it) && it < o->max_iters; ++k) {
      for (int64_t r = 0; r < mJ; ++r) yo[r] = D[r] * yp[r];
      orc_dual_grad(P, yo, gamma, gr, NULL, NULL);
      const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
      const double beta = (tk - 1.0) / tn;
      for (int64_t r = 0; r < mJ; ++r) {
        double step = yp[r] + eta * D[r] * gr[r]; /* ascent on the scaled dual */
        const int eq = (P->eq_mask >> (int)(r / J)) & 1;
        double ln = (eq || step > 0.0) ? step : 0.0; /* lam' >= 0 on inequality rows, free on equality rows */
        lo[r] = lp[r];
        lp[r] = ln;
        yp[r] = ln + beta * (ln - lo[r]);
      }
      tk = tn;
      ++it;
      while (snap < o->n_snap && o->snap_iters[snap] == it) {
        for (int64_t r = 0; r < mJ; ++r) o->snap_lambda[snap * mJ + r] = D[r] * lp[r];
        ++snap;
      }
      if (o->trace_dual) {
        for (int64_t r = 0; r < mJ; ++r) yo[r] = D[r] * lp[r];
        orc_dual_grad(P, yo, gamma, NULL, &o->trace_dual[it - 1], NULL);
      }
      if (last && o->check_every > 0 && (k + 1) % o->check_every == 0) {
        for (int64_t r = 0; r < mJ; ++r) yo[r] = D[r] * lp[r];
        orc_certificate(P, yo, gamma, &cs);
        cs.iters = it;
        cs.stage = s;
        if (cs.rel_gap <= o->tol) {
          cs.status = 0;
          done = 1;
          break;
        }
      }
    }
    if (it >= o->max_iters) break;
  }
  for (int64_t r = 0; r < mJ; ++r) lam_out[r] = D[r] * lp[r];
  if (!done) {
    orc_certificate(P, lam_out, o->gammas[o->n_stages - 1], &cs);
    cs.status = cs.rel_gap <= o->tol ? 0 : 1;
    cs.iters = it;
  }
  *st = cs;
  free(D); free(lp); free(yp); free(yo); free(gr); free(lo);
  return 0;
}
