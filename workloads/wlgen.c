/*
 * Seeded synthetic matching-LP instance generator.
 *
 * This module only produces input data (eligibility pattern, c, a); it holds
 * none of the solver's arithmetic and is shared by the CPU oracle and the GPU
 * path as their common source of inputs.
 *
 * Random numbers come from a counter-based Philox-4x32 generator with ten
 * rounds (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11).  Every user owns its own counter range, keyed by
 * (seed, stream), so an instance is bit-identical for any OpenMP thread count.
 *
 * The shape of the workloads follows the paper's matching setting (Section 3.3:
 * users x items, sparse eligibility, per-user simplex or box): per-user degree
 * distributions, item-popularity skew and value distributions are parameters.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10                                                            */
/* ------------------------------------------------------------------------ */
static void philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t x0 = in[0], x1 = in[1], x2 = in[2], x3 = in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Exposed for a known-answer test of the block function. */
void wl_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

typedef struct {
  uint32_t key[2];
  uint32_t ctr[4];
  uint32_t buf[4];
  int avail;
} rng_t;

/* One independent stream per (seed, stream id, entity). */
static void rng_init(rng_t* r, uint64_t seed, uint32_t stream, uint64_t entity) {
  r->key[0] = (uint32_t)seed;
  r->key[1] = stream;
  r->ctr[0] = (uint32_t)entity;
  r->ctr[1] = (uint32_t)(entity >> 32);
  r->ctr[2] = 0;
  r->ctr[3] = (uint32_t)(seed >> 32);
  r->avail = 0;
}

static uint32_t rng_u32(rng_t* r) {
  if (r->avail == 0) {
    philox4x32_10(r->ctr, r->key, r->buf);
    r->ctr[2]++;
    r->avail = 4;
  }
  return r->buf[4 - r->avail--];
}

/* Uniform on [0,1) with 53 random bits. */
static double rng_u01(rng_t* r) {
  uint64_t hi = rng_u32(r), lo = rng_u32(r);
  return (double)(((hi << 32) | lo) >> 11) * 0x1.0p-53;
}

/* Standard normal by the Box-Muller transform (one of the pair is used). */
static double rng_normal(rng_t* r) {
  double u1 = 1.0 - rng_u01(r); /* (0,1] */
  double u2 = rng_u01(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

/* Poisson by sequential inversion of the CDF (small means only). */
static int64_t rng_poisson(rng_t* r, double mean) {
  double u = rng_u01(r);
  double p = exp(-mean), F = p;
  int64_t k = 0;
  while (u > F && k < 100000) {
    ++k;
    p *= mean / (double)k;
    F += p;
  }
  return k;
}

/* ------------------------------------------------------------------------ */
/* Parameters                                                                */
/* ------------------------------------------------------------------------ */
enum { WL_DEG_POISSON = 0, WL_DEG_LOGNORMAL = 1, WL_DEG_CONST = 2 };
enum { WL_ITEM_UNIFORM = 0, WL_ITEM_ZIPF = 1 };
enum { WL_C_NEG_UNIFORM = 0, WL_C_NEG_UNIFORM_POP = 1 };
enum { WL_A_ONES = 0, WL_A_LOGNORMAL = 1 };

typedef struct {
  int64_t n_users;
  int32_t n_items;
  int32_t pad0;
  uint64_t seed;
  int32_t deg_kind;
  int32_t deg_min, deg_max;
  int32_t item_kind;
  double deg_p1, deg_p2; /* Poisson mean | lognormal (mu, sigma) | constant */
  double zipf_s;
  int32_t c_kind;
  int32_t n_families;
  int32_t a_kind[4];
  double a_p1[4], a_p2[4];
} wl_params;

/* stream ids */
#define S_DEG 1u
#define S_ITEM 2u
#define S_VAL 3u
#define S_PERM 7u
#define S_FAM 16u

static int64_t draw_degree(const wl_params* p, int64_t user) {
  rng_t r;
  rng_init(&r, p->seed, S_DEG, (uint64_t)user);
  int64_t d;
  if (p->deg_kind == WL_DEG_POISSON) {
    d = rng_poisson(&r, p->deg_p1);
  } else if (p->deg_kind == WL_DEG_LOGNORMAL) {
    double x = exp(p->deg_p1 + p->deg_p2 * rng_normal(&r));
    d = (int64_t)llround(x > 1e12 ? 1e12 : x);
  } else {
    d = (int64_t)p->deg_p1;
  }
  int64_t lo = p->deg_min, hi = p->deg_max;
  if (hi > p->n_items) hi = p->n_items;
  if (d < lo) d = lo;
  if (d > hi) d = hi;
  return d;
}

/* Fills row_ptr[0..I]; returns 0 on success. */
int wl_degrees(const wl_params* p, int64_t* row_ptr) {
  if (!p || !row_ptr || p->n_users < 0 || p->n_items <= 0) return -1;
  const int64_t I = p->n_users;
  int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)(I > 0 ? I : 1));
  if (!deg) return -2;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < I; ++i) deg[i] = draw_degree(p, i);
  row_ptr[0] = 0;
  for (int64_t i = 0; i < I; ++i) row_ptr[i + 1] = row_ptr[i] + deg[i];
  free(deg);
  return 0;
}

/* Popularity rank (0 = most popular) of each item id, from a seeded
 * Fisher-Yates shuffle; rank_of[item] = rank. */
static void item_ranks(const wl_params* p, int32_t* rank_of) {
  const int32_t J = p->n_items;
  int32_t* item_at = (int32_t*)malloc(sizeof(int32_t) * (size_t)J);
  for (int32_t j = 0; j < J; ++j) item_at[j] = j;
  rng_t r;
  rng_init(&r, p->seed, S_PERM, 0);
  for (int32_t j = J - 1; j > 0; --j) {
    int32_t t = (int32_t)(rng_u01(&r) * (double)(j + 1));
    if (t > j) t = j;
    int32_t tmp = item_at[j]; item_at[j] = item_at[t]; item_at[t] = tmp;
  }
  for (int32_t rank = 0; rank < J; ++rank) rank_of[item_at[rank]] = rank;
  free(item_at);
}

/* Fenwick tree (1-based internally) over J integer weights. */
static void fenwick_add(uint64_t* fw, int32_t J, int32_t k, uint64_t delta) {
  for (int32_t i = k + 1; i <= J; i += i & (-i)) fw[i] += delta;
}

/* Smallest 0-based k with prefix sum (w_0 + ... + w_k) > t. */
static int32_t fenwick_find(const uint64_t* fw, int32_t J, uint64_t t) {
  int32_t pos = 0, step = 1;
  while (step * 2 <= J) step *= 2;
  for (; step > 0; step >>= 1) {
    if (pos + step <= J && fw[pos + step] <= t) {
      pos += step;
      t -= fw[pos];
    }
  }
  return pos;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static void sort_row(int32_t* v, int64_t d) {
  if (d < 32) {
    for (int64_t i = 1; i < d; ++i) {
      int32_t x = v[i];
      int64_t k = i - 1;
      while (k >= 0 && v[k] > x) { v[k + 1] = v[k]; --k; }
      v[k + 1] = x;
    }
  } else {
    qsort(v, (size_t)d, sizeof(int32_t), cmp_i32);
  }
}

/*
 * Fills the rows given row_ptr (from wl_degrees).
 *   item_idx[nnz]            eligible items, strictly increasing per row
 *   c[nnz]                   value coefficients
 *   a_out[n_lognormal * nnz] coefficients of the non-ones families, in family order
 *   item_weight[J]           popularity weight (rank+1)^-s per item (nullable)
 */
int wl_fill(const wl_params* p, const int64_t* row_ptr, int32_t* item_idx, float* c,
            float* a_out, double* item_weight) {
  if (!p || !row_ptr || !item_idx || !c) return -1;
  const int64_t I = p->n_users;
  const int32_t J = p->n_items;
  int32_t* rank_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)J);
  int32_t* item_at = (int32_t*)malloc(sizeof(int32_t) * (size_t)J);
  double* weight = (double*)malloc(sizeof(double) * (size_t)J);
  item_ranks(p, rank_of);
  for (int32_t j = 0; j < J; ++j) {
    item_at[rank_of[j]] = j;
    weight[j] = pow((double)(rank_of[j] + 1), -p->zipf_s);
  }
  if (item_weight) memcpy(item_weight, weight, sizeof(double) * (size_t)J);
  uint64_t* wint = NULL;
  uint64_t* fw_base = NULL;
  uint64_t fw_total = 0;
  if (p->item_kind == WL_ITEM_ZIPF) {
    wint = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)J);
    fw_base = (uint64_t*)calloc((size_t)J + 1, sizeof(uint64_t));
    for (int32_t k = 0; k < J; ++k) {
      wint[k] = (uint64_t)llround(ldexp(pow((double)(k + 1), -p->zipf_s), 44));
      if (wint[k] == 0) wint[k] = 1;
      fw_total += wint[k];
      fenwick_add(fw_base, J, k, wint[k]);
    }
  }
  const int64_t nnz = row_ptr[I];
  const size_t words = ((size_t)J + 63) / 64;
  int failed = 0;

#pragma omp parallel
  {
    uint64_t* seen = (uint64_t*)calloc(words, sizeof(uint64_t));
    uint64_t* fw = NULL;
    int32_t* taken = NULL;
    if (p->item_kind == WL_ITEM_ZIPF) {
      fw = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)J + 1));
      memcpy(fw, fw_base, sizeof(uint64_t) * ((size_t)J + 1));
      taken = (int32_t*)malloc(sizeof(int32_t) * (size_t)J);
    }
#pragma omp for schedule(dynamic, 1024)
    for (int64_t i = 0; i < I; ++i) {
      const int64_t s = row_ptr[i];
      const int64_t d = row_ptr[i + 1] - s;
      int32_t* row = item_idx + s;
      rng_t r;
      rng_init(&r, p->seed, S_ITEM, (uint64_t)i);
      if (d > J) { failed = 1; continue; }
      if (p->item_kind == WL_ITEM_UNIFORM) {
        /* Floyd's sampling of d distinct items out of J */
        int64_t n = 0;
        for (int64_t jj = J - d; jj < J; ++jj) {
          int64_t t = (int64_t)(rng_u01(&r) * (double)(jj + 1));
          if (t > jj) t = jj;
          if (seen[t >> 6] & (1ull << (t & 63))) t = jj;
          seen[t >> 6] |= 1ull << (t & 63);
          row[n++] = (int32_t)t;
        }
      } else {
        /* Successive sampling without replacement, proportional to the Zipf
         * weight of the items not yet taken (the same law as redrawing
         * duplicates).  An integer Fenwick tree over ranks holds the remaining
         * weights; taken ranks are restored afterwards, exactly. */
        uint64_t remaining = fw_total;
        for (int64_t n = 0; n < d; ++n) {
          uint64_t t = (uint64_t)(rng_u01(&r) * (double)remaining);
          if (t >= remaining) t = remaining - 1;
          int32_t rank = fenwick_find(fw, J, t);
          fenwick_add(fw, J, rank, (uint64_t)0 - wint[rank]);
          remaining -= wint[rank];
          taken[n] = rank;
          int32_t it = item_at[rank];
          seen[it >> 6] |= 1ull << (it & 63);
          row[n] = it;
        }
        for (int64_t n = 0; n < d; ++n) fenwick_add(fw, J, taken[n], wint[taken[n]]);
      }
      if ((size_t)d * 4 >= words) {
        /* rows are emitted in increasing item order straight from the bitmap */
        int64_t n = 0;
        for (size_t wd = 0; wd < words; ++wd) {
          uint64_t bits = seen[wd];
          while (bits) {
            int b = __builtin_ctzll(bits);
            row[n++] = (int32_t)(wd * 64 + (size_t)b);
            bits &= bits - 1;
          }
          seen[wd] = 0;
        }
      } else {
        for (int64_t e = 0; e < d; ++e) seen[row[e] >> 6] &= ~(1ull << (row[e] & 63));
        sort_row(row, d);
      }
      /* values in row order, from the user's own value stream */
      rng_t rv;
      rng_init(&rv, p->seed, S_VAL, (uint64_t)i);
      for (int64_t e = 0; e < d; ++e) {
        double u = rng_u01(&rv);
        double val = (p->c_kind == WL_C_NEG_UNIFORM_POP) ? -u * weight[row[e]] : -u;
        c[s + e] = (float)val;
      }
      int64_t stored = 0;
      for (int32_t k = 0; k < p->n_families && k < 4; ++k) {
        if (p->a_kind[k] != WL_A_LOGNORMAL) continue;
        rng_t ra;
        rng_init(&ra, p->seed, S_FAM + (uint32_t)k, (uint64_t)i);
        float* dst = a_out + stored * nnz + s;
        for (int64_t e = 0; e < d; ++e) dst[e] = (float)exp(p->a_p1[k] + p->a_p2[k] * rng_normal(&ra));
        ++stored;
      }
    }
    free(seen);
    free(fw);
    free(taken);
  }
  free(rank_of); free(item_at); free(weight); free(wint); free(fw_base);
  return failed ? -3 : 0;
}

/* ------------------------------------------------------------------------ */
/* The paper's Appendix-A construction                                       */
/* ------------------------------------------------------------------------ */
/* Resource-major generation (Appendix A): every resource (item) j draws a
 * lognormal breadth, its share p_j of the total breadth sets the number of
 * incident requests (users) K_j ~ Poisson(p_j I nu) truncated at I, and it
 * picks K_j distinct users.  Edge value c_ij = min(v_j u_i eps_ij, c_max)
 * (v, u, eps lognormal), coefficient a_ij = s_j c_ij (s lognormal), capacity
 * b_j = rho_j (l_j + eps0) with l_j the greedy load (each user gives its
 * largest a_ij to that resource) and rho_j ~ U[0.5, 1].  The paper leaves the
 * distribution parameters open; they are arguments here. */
typedef struct {
  int64_t n_users;
  int32_t n_items;
  int32_t pad0;
  uint64_t seed;
  double nu;            /* mean nonzeros per user */
  double breadth_sigma; /* log-sd of the resource breadth */
  double value_sigma;   /* log-sd of v_j */
  double resp_sigma;    /* log-sd of u_i */
  double noise_sigma;   /* log-sd of eps_ij */
  double c_max;         /* cap of the edge value */
  double scale_sigma;   /* log-sd of s_j */
  double eps0;          /* added to the greedy load */
} wl_appx_params;

#define S_APPX_BREADTH 40u
#define S_APPX_COUNT 41u
#define S_APPX_PICK 42u
#define S_APPX_VJ 43u
#define S_APPX_UI 44u
#define S_APPX_EDGE 45u
#define S_APPX_SJ 46u
#define S_APPX_RHO 47u

/* Poisson count: inversion for small means, else the normal approximation
 * round(mean + sqrt(mean) N(0,1)) clipped at 0. */
static int64_t appx_poisson(rng_t* r, double mean) {
  if (mean < 100.0) return rng_poisson(r, mean);
  double x = mean + sqrt(mean) * rng_normal(r);
  return x < 0.0 ? 0 : (int64_t)llround(x);
}

/* K[j] for every resource; returns the number of edges (or < 0). */
int64_t wl_appx_counts(const wl_appx_params* p, int64_t* K) {
  if (!p || !K || p->n_users <= 0 || p->n_items <= 0) return -1;
  const int32_t J = p->n_items;
  double* w = (double*)malloc(sizeof(double) * (size_t)J);
  if (!w) return -2;
  double tot = 0.0;
  for (int32_t j = 0; j < J; ++j) {
    rng_t r;
    rng_init(&r, p->seed, S_APPX_BREADTH, (uint64_t)j);
    w[j] = exp(p->breadth_sigma * rng_normal(&r));
    tot += w[j];
  }
  int64_t nnz = 0;
  for (int32_t j = 0; j < J; ++j) {
    rng_t r;
    rng_init(&r, p->seed, S_APPX_COUNT, (uint64_t)j);
    int64_t k = appx_poisson(&r, w[j] / tot * (double)p->n_users * p->nu);
    if (k > p->n_users) k = p->n_users;
    K[j] = k;
    nnz += k;
  }
  free(w);
  return nnz;
}

typedef struct {
  int32_t item;
  float c, a;
} appx_edge;

static int cmp_edge(const void* x, const void* y) {
  const int32_t a = ((const appx_edge*)x)->item, b = ((const appx_edge*)y)->item;
  return (a > b) - (a < b);
}

/* Fills the user-major CSR (rows sorted by item), c (the value, >= 0), a and b. */
int wl_appx_fill(const wl_appx_params* p, const int64_t* K, int64_t* row_ptr, int32_t* item_idx, float* c,
                 float* a, double* b) {
  if (!p || !K || !row_ptr || !item_idx || !c || !a || !b) return -1;
  const int64_t I = p->n_users;
  const int32_t J = p->n_items;
  int64_t* kofs = (int64_t*)malloc(sizeof(int64_t) * ((size_t)J + 1));
  kofs[0] = 0;
  for (int32_t j = 0; j < J; ++j) kofs[j + 1] = kofs[j] + K[j];
  const int64_t nnz = kofs[J];
  int32_t* user_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  float* cv = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
  double* ui = (double*)malloc(sizeof(double) * (size_t)I);
  int64_t* deg = (int64_t*)calloc((size_t)I + 1, sizeof(int64_t));
  double* sj = (double*)malloc(sizeof(double) * (size_t)J);
  if (!kofs || !user_of || !cv || !ui || !deg || !sj) return -2;
  if (I > 2147483647LL) return -4;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < I; ++i) {
    rng_t r;
    rng_init(&r, p->seed, S_APPX_UI, (uint64_t)i);
    ui[i] = exp(p->resp_sigma * rng_normal(&r));
  }
  for (int32_t j = 0; j < J; ++j) {
    rng_t r;
    rng_init(&r, p->seed, S_APPX_SJ, (uint64_t)j);
    sj[j] = exp(p->scale_sigma * rng_normal(&r));
  }
  const size_t words = ((size_t)I + 63) / 64;
#pragma omp parallel
  {
    uint64_t* seen = (uint64_t*)calloc(words, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 1)
    for (int32_t j = 0; j < J; ++j) {
      int32_t* lst = user_of + kofs[j];
      const int64_t k = K[j];
      rng_t r;
      rng_init(&r, p->seed, S_APPX_PICK, (uint64_t)j);
      if (2 * k <= I) {
        /* distinct users by redrawing repeats */
        for (int64_t n = 0; n < k;) {
          int64_t t = (int64_t)(rng_u01(&r) * (double)I);
          if (t >= I) t = I - 1;
          if (seen[t >> 6] & (1ull << (t & 63))) continue;
          seen[t >> 6] |= 1ull << (t & 63);
          lst[n++] = (int32_t)t;
        }
        for (int64_t n = 0; n < k; ++n) seen[lst[n] >> 6] &= ~(1ull << (lst[n] & 63));
      } else {
        /* Floyd's sampling for dense resources */
        int64_t n = 0;
        for (int64_t jj = I - k; jj < I; ++jj) {
          int64_t t = (int64_t)(rng_u01(&r) * (double)(jj + 1));
          if (t > jj) t = jj;
          if (seen[t >> 6] & (1ull << (t & 63))) t = jj;
          seen[t >> 6] |= 1ull << (t & 63);
          lst[n++] = (int32_t)t;
        }
        for (int64_t e = 0; e < k; ++e) seen[lst[e] >> 6] &= ~(1ull << (lst[e] & 63));
      }
      rng_t rv, re;
      rng_init(&rv, p->seed, S_APPX_VJ, (uint64_t)j);
      const double vj = exp(p->value_sigma * rng_normal(&rv));
      rng_init(&re, p->seed, S_APPX_EDGE, (uint64_t)j);
      for (int64_t n = 0; n < k; ++n) {
        double val = vj * ui[lst[n]] * exp(p->noise_sigma * rng_normal(&re));
        cv[kofs[j] + n] = (float)(val < p->c_max ? val : p->c_max);
      }
    }
    free(seen);
  }
  /* user-major transpose: counts, offsets, scatter, then each row sorted by item */
  for (int64_t e = 0; e < nnz; ++e) deg[user_of[e]]++;
  row_ptr[0] = 0;
  for (int64_t i = 0; i < I; ++i) row_ptr[i + 1] = row_ptr[i] + deg[i];
  appx_edge* ed = (appx_edge*)malloc(sizeof(appx_edge) * (size_t)(nnz > 0 ? nnz : 1));
  for (int64_t i = 0; i < I; ++i) deg[i] = row_ptr[i];
  for (int32_t j = 0; j < J; ++j)
    for (int64_t n = kofs[j]; n < kofs[j + 1]; ++n) {
      const int32_t u = user_of[n];
      appx_edge x = {j, cv[n], (float)(sj[j] * (double)cv[n])};
      ed[deg[u]++] = x;
    }
  double* load = (double*)calloc((size_t)J, sizeof(double));
  int32_t* best_j = (int32_t*)malloc(sizeof(int32_t) * (size_t)I);
  float* best_a = (float*)malloc(sizeof(float) * (size_t)I);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < I; ++i) {
    const int64_t s0 = row_ptr[i], d = row_ptr[i + 1] - s0;
    if (d > 1) qsort(ed + s0, (size_t)d, sizeof(appx_edge), cmp_edge);
    int32_t bj = -1;
    float ba = -1.f;
    for (int64_t e = 0; e < d; ++e) {
      item_idx[s0 + e] = ed[s0 + e].item;
      c[s0 + e] = ed[s0 + e].c;
      a[s0 + e] = ed[s0 + e].a;
      if (ed[s0 + e].a > ba) {
        ba = ed[s0 + e].a;
        bj = ed[s0 + e].item;
      }
    }
    best_j[i] = bj;
    best_a[i] = ba;
  }
  /* greedy loads, summed in user order */
  for (int64_t i = 0; i < I; ++i)
    if (best_j[i] >= 0) load[best_j[i]] += (double)best_a[i];
  for (int32_t j = 0; j < J; ++j) {
    rng_t r;
    rng_init(&r, p->seed, S_APPX_RHO, (uint64_t)j);
    b[j] = (0.5 + 0.5 * rng_u01(&r)) * (load[j] + p->eps0);
  }
  free(kofs); free(user_of); free(cv); free(ui); free(deg); free(sj); free(ed); free(load); free(best_j);
  free(best_a);
  return 0;
}

/* Uniform and normal draws for drift and other per-element perturbations:
 * out[n] for entities [first, first+n) on the given stream. kind 0: U[0,1),
 * kind 1: N(0,1). */
int wl_draw(uint64_t seed, uint32_t stream, int64_t first, int64_t n, int kind, double* out) {
  if (!out || n < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < n; ++e) {
    rng_t r;
    rng_init(&r, seed, stream, (uint64_t)(first + e));
    out[e] = (kind == 0) ? rng_u01(&r) : rng_normal(&r);
  }
  return 0;
}
