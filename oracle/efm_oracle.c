/*
 * efm_oracle.c -- plain CPU oracle of the exhaustive AND/OR pathway traversal.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares nothing with the
 * GPU library (no headers, helpers or tables) and is deliberately slow and
 * literal: every child is classified with an exact rank computation, every
 * level is a sorted set, no shortcut is taken.
 *
 * What it computes (paper, Section 2.1, Definitions 1-3; Section 3.1,
 * Definitions 8-9; Section 4.1, INIT and Algorithm 3 made exhaustive as in the
 * proof of Theorem 1, Section 5.3):
 *
 *   Given S (m x n integers), reversibility flags, external flags, a target
 *   external metabolite x and a depth cap D, emit every pair (E, v) with
 *     - v an integer vector with gcd 1 and supp(v) = E, |E| <= D,
 *     - S_int v = 0 over the internal rows (Definition 2, steady state),
 *     - v_r > 0 for every irreversible r in E (Definition 2),
 *     - S[x,:] v > 0 (the pathway produces the target; INIT seeds the target
 *       reaction with a positive flux),
 *     - no flux-balanced v' with supp(v') strictly inside E (Definition 3).
 *
 * The traversal (level k holds reaction sets of size k):
 *   level 1: { {t} } for every reaction t that can produce x;
 *   a partial pathway P is expanded at its lowest-index internal metabolite that
 *   is touched but not balanced topologically (one-sided, or touched once):
 *   the forward flow (Definition 9) adds a consumer, the backward flow a
 *   producer, a lone reversible reaction any other reaction at that metabolite.
 *   If every touched metabolite is covered but P's columns are independent,
 *   any reaction touching a touched internal metabolite is added.
 *   A child whose columns are independent survives to the next level; a
 *   dependent child has a one-dimensional null space, and its null vector is
 *   emitted if it has full support, feasible signs and produces x; otherwise it
 *   is dropped (no superset can be elementary).
 *   Frontiers larger than a cap keep their smallest keys, reading a reaction
 *   set as an n-bit unsigned integer in which reaction r weighs 2^r.
 *
 * Arithmetic: exact, fraction-free Bareiss elimination over __int128 with
 * overflow checks on every operation.  An overflow aborts with an error code.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_EOVERFLOW -4

#define ORC_COMPLETE 0u
#define ORC_DEPTH_CAPPED 1u
#define ORC_FRONTIER_TRUNCATED 2u

#define ORC_MAXK 128            /* largest support size handled */

typedef struct {
  int m, n, W;          /* metabolites, reactions, 64-bit words per reaction set */
  const int32_t *S;     /* row-major m x n */
  const uint8_t *rev;   /* n */
  const uint8_t *ext;   /* m */
} net_t;

typedef struct {
  uint64_t *keys;       /* count x W */
  int64_t count, cap;
} keyset_t;

/* per-level counters reported for parity checks */
typedef struct {
  int64_t parents, children, unique, independent, emitted, kept;
} orc_level_t;

static int g_overflow;

/* ------------------------------------------------------------ checked int128 */
static i128 cmul(i128 a, i128 b) {
  i128 r;
  if (__builtin_mul_overflow(a, b, &r)) { g_overflow = 1; return 0; }
  return r;
}
static i128 csub(i128 a, i128 b) {
  i128 r;
  if (__builtin_sub_overflow(a, b, &r)) { g_overflow = 1; return 0; }
  return r;
}
static i128 cadd(i128 a, i128 b) {
  i128 r;
  if (__builtin_add_overflow(a, b, &r)) { g_overflow = 1; return 0; }
  return r;
}
static i128 iabs128(i128 a) { return a < 0 ? -a : a; }
static i128 gcd128(i128 a, i128 b) {
  a = iabs128(a); b = iabs128(b);
  while (b) { i128 t = a % b; a = b; b = t; }
  return a;
}

/* ------------------------------------------------------------ reaction sets */
static int has(const uint64_t *P, int r) { return (int)((P[r >> 6] >> (r & 63)) & 1u); }
static void put(uint64_t *P, int r) { P[r >> 6] |= (uint64_t)1 << (r & 63); }
static int popcount_set(const uint64_t *P, int W) {
  int c = 0;
  for (int w = 0; w < W; ++w) c += __builtin_popcountll(P[w]);
  return c;
}
/* canonical order: the set read as an unsigned integer, reaction r weighs 2^r */
static int g_W_cmp;
static int key_cmp(const void *a, const void *b) {
  const uint64_t *x = (const uint64_t *)a, *y = (const uint64_t *)b;
  for (int w = g_W_cmp - 1; w >= 0; --w) {
    if (x[w] < y[w]) return -1;
    if (x[w] > y[w]) return 1;
  }
  return 0;
}

static int keyset_push(keyset_t *ks, const uint64_t *key, int W) {
  if (ks->count == ks->cap) {
    int64_t nc = ks->cap ? ks->cap * 2 : 1024;
    uint64_t *nk = (uint64_t *)realloc(ks->keys, (size_t)nc * W * sizeof(uint64_t));
    if (!nk) return ORC_ENOMEM;
    ks->keys = nk;
    ks->cap = nc;
  }
  memcpy(ks->keys + (size_t)ks->count * W, key, (size_t)W * sizeof(uint64_t));
  ks->count++;
  return ORC_OK;
}

static void keyset_sort_unique(keyset_t *ks, int W) {
  if (ks->count == 0) return;
  g_W_cmp = W;
  qsort(ks->keys, (size_t)ks->count, (size_t)W * sizeof(uint64_t), key_cmp);
  int64_t out = 1;
  for (int64_t i = 1; i < ks->count; ++i) {
    if (key_cmp(ks->keys + (size_t)i * W, ks->keys + (size_t)(out - 1) * W) != 0) {
      if (out != i) memcpy(ks->keys + (size_t)out * W, ks->keys + (size_t)i * W, (size_t)W * 8);
      out++;
    }
  }
  ks->count = out;
}

/* ------------------------------------------------ topological roles (Defs 8-10)
 * For every internal metabolite i and the partial pathway P:
 *   a[i] = irreversible reactions of P producing i, b[i] = irreversible reactions
 *   of P consuming i, c[i] = reversible reactions of P touching i. */
static void roles(const net_t *N, const uint64_t *P, int *a, int *b, int *c) {
  for (int i = 0; i < N->m; ++i) a[i] = b[i] = c[i] = 0;
  for (int r = 0; r < N->n; ++r) {
    if (!has(P, r)) continue;
    for (int i = 0; i < N->m; ++i) {
      int32_t s = N->S[(size_t)i * N->n + r];
      if (s == 0 || N->ext[i]) continue;
      if (N->rev[r]) c[i]++;
      else if (s > 0) a[i]++;
      else b[i]++;
    }
  }
}

/* touched: some reaction of P involves i.  covered: i has a possible producer and
 * a possible consumer among two or more reactions of P (a metabolite touched once,
 * or only from one side, cannot be balanced -- Eq. 2's extra flux is nonzero). */
static int touched(int a, int b, int c) { return a + b + c >= 1; }
static int covered(int a, int b, int c) {
  return (a >= 1 || c >= 1) && (b >= 1 || c >= 1) && (a + b + c >= 2);
}

/* Children of P (Algorithm 3's branch over the outputs/inputs of the chosen
 * metabolite, every branch taken).  Writes candidate reactions into cand[],
 * returns their count.  a, b, c are scratch arrays of m ints. */
static int expand(const net_t *N, const uint64_t *P, int *cand, int *a, int *b, int *c) {
  int m = N->m, n = N->n;
  roles(N, P, a, b, c);
  int istar = -1;
  for (int i = 0; i < m && istar < 0; ++i)
    if (!N->ext[i] && touched(a[i], b[i], c[i]) && !covered(a[i], b[i], c[i])) istar = i;
  int k = 0;
  if (istar >= 0) {
    int ia = a[istar], ib = b[istar], ic = c[istar];
    for (int r = 0; r < n; ++r) {
      if (has(P, r)) continue;
      int32_t s = N->S[(size_t)istar * n + r];
      if (s == 0) continue;
      int ok;
      if (ic == 1 && ia == 0 && ib == 0) ok = 1;              /* lone reversible: any */
      else if (ia >= 1) ok = N->rev[r] || s < 0;              /* forward: a consumer */
      else ok = N->rev[r] || s > 0;                           /* backward: a producer */
      if (ok) cand[k++] = r;
    }
  } else {
    /* closed: every reaction touching an internal metabolite that P touches */
    for (int r = 0; r < n; ++r) {
      if (has(P, r)) continue;
      int hit = 0;
      for (int i = 0; i < m && !hit; ++i)
        if (!N->ext[i] && N->S[(size_t)i * n + r] != 0 && touched(a[i], b[i], c[i])) hit = 1;
      if (hit) cand[k++] = r;
    }
  }
  return k;
}

/* ----------------------------------------- exact null space of S_int[:, Q]
 * Fraction-free Gaussian elimination (Bareiss) of the internal-row submatrix on
 * the columns of Q.  Returns the rank; if rank == |Q|-1 the primitive integer
 * null vector (gcd 1, first nonzero entry positive) is written to v[0..k-1] in
 * column order of cols[]. */
static int null_space(const net_t *N, const int *cols, int k, i128 *v, i128 *work) {
  int m = N->m, n = N->n;
  int rows = 0;
  i128 *A = work;                      /* rows x k, rows <= m */
  for (int i = 0; i < m; ++i) {
    if (N->ext[i]) continue;
    int nz = 0;
    for (int j = 0; j < k; ++j) nz |= N->S[(size_t)i * n + cols[j]] != 0;
    if (!nz) continue;
    for (int j = 0; j < k; ++j) A[(size_t)rows * k + j] = N->S[(size_t)i * n + cols[j]];
    rows++;
  }
  int pivcol[ORC_MAXK];
  int rank = 0;
  i128 prev = 1;
  for (int col = 0; col < k && rank < rows; ++col) {
    int piv = -1;
    for (int i = rank; i < rows; ++i)
      if (A[(size_t)i * k + col] != 0) { piv = i; break; }
    if (piv < 0) continue;
    if (piv != rank)
      for (int j = 0; j < k; ++j) {
        i128 t = A[(size_t)piv * k + j];
        A[(size_t)piv * k + j] = A[(size_t)rank * k + j];
        A[(size_t)rank * k + j] = t;
      }
    i128 p = A[(size_t)rank * k + col];
    for (int i = rank + 1; i < rows; ++i) {
      i128 f = A[(size_t)i * k + col];
      for (int j = col; j < k; ++j) {
        /* Bareiss step: exact division by the previous pivot */
        i128 num = csub(cmul(p, A[(size_t)i * k + j]), cmul(f, A[(size_t)rank * k + j]));
        A[(size_t)i * k + j] = num / prev;
      }
      if (g_overflow) return -1;
    }
    pivcol[rank] = col;
    prev = p;
    rank++;
  }
  if (rank != k - 1 || g_overflow) return rank;
  /* the single free column */
  int isfree[ORC_MAXK] = {0};
  for (int j = 0; j < k; ++j) isfree[j] = 1;
  for (int t = 0; t < rank; ++t) isfree[pivcol[t]] = 0;
  int f = -1;
  for (int j = 0; j < k; ++j) if (isfree[j]) f = j;
  /* integer back substitution, v_f = 1: row t gives
   * U[t][pc] v_pc + sum_{j > pc} U[t][j] v_j = 0.  When U[t][pc] does not divide the
   * sum, every entry set so far is scaled up first; the partial vector is kept
   * primitive, so its entries never exceed those of the final null vector. */
  for (int j = 0; j < k; ++j) v[j] = 0;
  v[f] = 1;
  for (int t = rank - 1; t >= 0; --t) {
    int pc = pivcol[t];
    i128 sum = 0;
    for (int j = pc + 1; j < k; ++j)
      if (v[j] != 0 && A[(size_t)t * k + j] != 0)
        sum = cadd(sum, cmul(A[(size_t)t * k + j], v[j]));
    i128 p = A[(size_t)t * k + pc];
    i128 g = gcd128(sum, p);             /* g >= 1 since p != 0 */
    i128 mult = iabs128(p) / g;
    if (mult != 1)
      for (int j = pc + 1; j < k; ++j) v[j] = cmul(v[j], mult);
    v[pc] = (p > 0) ? -(sum / g) : (sum / g);
    if (g_overflow) return -1;
    i128 G = 0;
    for (int j = pc; j < k; ++j) G = gcd128(G, v[j]);
    if (G > 1) for (int j = pc; j < k; ++j) v[j] /= G;
  }
  int first = -1;
  for (int j = 0; j < k && first < 0; ++j) if (v[j] != 0) first = j;
  if (first >= 0 && v[first] < 0) for (int j = 0; j < k; ++j) v[j] = -v[j];
  return rank;
}

/* ------------------------------------------------------------------- driver */
typedef struct {
  keyset_t found_keys;
  int64_t *found_flux;   /* dense n per found pathway */
  int64_t found_count, found_cap;
} found_t;

static int found_push(found_t *F, const uint64_t *key, const int64_t *flux, int W, int n) {
  int rc = keyset_push(&F->found_keys, key, W);
  if (rc) return rc;
  if (F->found_count == F->found_cap) {
    int64_t nc = F->found_cap ? F->found_cap * 2 : 1024;
    int64_t *nf = (int64_t *)realloc(F->found_flux, (size_t)nc * n * sizeof(int64_t));
    if (!nf) return ORC_ENOMEM;
    F->found_flux = nf;
    F->found_cap = nc;
  }
  memcpy(F->found_flux + (size_t)F->found_count * n, flux, (size_t)n * sizeof(int64_t));
  F->found_count++;
  return ORC_OK;
}

typedef struct orc_result {
  int W, n;
  uint32_t status;
  int64_t count;
  uint64_t *keys;
  int64_t *flux;
  int n_levels;
  orc_level_t levels[1100];
} orc_result;

/* Classify one child Q: returns 1 = independent, 2 = emitted (flux written),
 * 0 = dropped; negative on error. */
static int classify(const net_t *N, const uint64_t *Q, int x, int64_t *flux_out,
                    i128 *work, i128 *v) {
  int n = N->n;
  int cols[1024];
  int k = 0;
  for (int r = 0; r < n; ++r) if (has(Q, r)) cols[k++] = r;
  if (k > ORC_MAXK) return ORC_EINVAL;
  int rank = null_space(N, cols, k, v, work);
  if (g_overflow) return ORC_EOVERFLOW;
  if (rank == k) return 1;
  if (rank < k - 1) return 0;           /* cannot happen for an independent parent */
  /* full support */
  for (int j = 0; j < k; ++j) if (v[j] == 0) return 0;
  /* sign feasibility: all irreversible entries share one sign, which becomes + */
  int sgn = 0;
  for (int j = 0; j < k; ++j) {
    if (N->rev[cols[j]]) continue;
    int s = v[j] > 0 ? 1 : -1;
    if (sgn == 0) sgn = s;
    else if (s != sgn) return 0;
  }
  /* target production S[x,:] v */
  i128 prod = 0;
  for (int j = 0; j < k; ++j)
    prod = cadd(prod, cmul((i128)N->S[(size_t)x * n + cols[j]], v[j]));
  if (g_overflow) return ORC_EOVERFLOW;
  if (sgn == 0) sgn = prod > 0 ? 1 : -1;   /* all reversible: orient to produce x */
  if (sgn < 0) { prod = -prod; for (int j = 0; j < k; ++j) v[j] = -v[j]; }
  if (prod <= 0) return 0;
  memset(flux_out, 0, (size_t)n * sizeof(int64_t));
  for (int j = 0; j < k; ++j) {
    if (v[j] > INT64_MAX || v[j] < INT64_MIN) return ORC_EOVERFLOW;
    flux_out[cols[j]] = (int64_t)v[j];
  }
  return 2;
}

/* One level: G holds the generated children (with repeats).  They are made a set,
 * each is classified, independent ones below the depth cap form the next
 * frontier (truncated to its smallest keys past the frontier cap), emitted ones
 * join the found list. */
static int settle(const net_t *N, keyset_t *G, int x, int D, int64_t frontier_cap,
                  orc_level_t *L, keyset_t *next, found_t *F, uint32_t *status,
                  i128 *work, i128 *v, int64_t *flux) {
  int W = N->W, rc;
  keyset_sort_unique(G, W);
  L->unique = G->count;
  next->count = 0;
  int depth_dropped = 0;
  for (int64_t q = 0; q < G->count; ++q) {
    const uint64_t *Q = G->keys + (size_t)q * W;
    int c = classify(N, Q, x, flux, work, v);
    if (c < 0) return c;
    if (c == 1) {
      L->independent++;
      if (popcount_set(Q, W) < D) {
        if ((rc = keyset_push(next, Q, W))) return rc;
      } else {
        depth_dropped = 1;
      }
    } else if (c == 2) {
      L->emitted++;
      if ((rc = found_push(F, Q, flux, W, N->n))) return rc;
    }
  }
  if (depth_dropped) *status |= ORC_DEPTH_CAPPED;
  /* next is sorted already: a subsequence of the sorted G */
  if (frontier_cap > 0 && next->count > frontier_cap) {
    next->count = frontier_cap;
    *status |= ORC_FRONTIER_TRUNCATED;
  }
  L->kept = next->count;
  return ORC_OK;
}

/* orc_enumerate: see the file header.  depth_cap <= 0 means no cap (n);
 * frontier_cap <= 0 means no cap.  On success *out owns the result. */
int orc_enumerate(int m, int n, const int32_t *S, const uint8_t *rev, const uint8_t *ext,
                  int x, int depth_cap, int64_t frontier_cap, orc_result **out) {
  if (!S || !rev || !ext || !out || m <= 0 || n <= 0 || n > 1024 || x < 0 || x >= m || !ext[x])
    return ORC_EINVAL;
  net_t N = {m, n, (n + 63) / 64, S, rev, ext};
  int W = N.W;
  int D = depth_cap > 0 && depth_cap < n ? depth_cap : n;
  if (D > ORC_MAXK) D = ORC_MAXK;           /* larger supports are not handled */
  g_overflow = 0;

  orc_result *R = (orc_result *)calloc(1, sizeof(orc_result));
  if (!R) return ORC_ENOMEM;
  R->W = W; R->n = n;
  found_t F;
  memset(&F, 0, sizeof(F));
  keyset_t cur = {0}, nxt = {0};
  uint64_t *key = (uint64_t *)calloc((size_t)W, sizeof(uint64_t));
  i128 *work = (i128 *)malloc((size_t)m * ORC_MAXK * sizeof(i128));
  int64_t *flux = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int *cand = (int *)malloc((size_t)n * sizeof(int));
  int *ra = (int *)malloc((size_t)m * 3 * sizeof(int));
  i128 v[ORC_MAXK];
  int rc = ORC_OK;
  if (!key || !work || !flux || !cand || !ra) { rc = ORC_ENOMEM; goto done; }

  /* INIT: every reaction that can produce x starts a pathway (level 1) */
  {
    keyset_t G = {0};
    for (int r = 0; r < n; ++r) {
      int32_t s = S[(size_t)x * n + r];
      if (s > 0 || (s < 0 && rev[r])) {
        memset(key, 0, (size_t)W * 8);
        put(key, r);
        if ((rc = keyset_push(&G, key, W))) { free(G.keys); goto done; }
      }
    }
    R->levels[0].children = G.count;
    rc = settle(&N, &G, x, D, frontier_cap, &R->levels[0], &cur, &F, &R->status, work, v, flux);
    free(G.keys);
    if (rc) goto done;
    R->n_levels = 1;
  }

  for (int k = 1; k <= D - 1 && cur.count > 0; ++k) {
    keyset_t G = {0};
    orc_level_t *L = &R->levels[k];
    L->parents = cur.count;
    for (int64_t p = 0; p < cur.count; ++p) {
      const uint64_t *P = cur.keys + (size_t)p * W;
      int nc = expand(&N, P, cand, ra, ra + m, ra + 2 * m);
      for (int c = 0; c < nc; ++c) {
        memcpy(key, P, (size_t)W * 8);
        put(key, cand[c]);
        if ((rc = keyset_push(&G, key, W))) { free(G.keys); goto done; }
      }
      L->children += nc;
    }
    rc = settle(&N, &G, x, D, frontier_cap, L, &nxt, &F, &R->status, work, v, flux);
    free(G.keys);
    if (rc) goto done;
    R->n_levels = k + 1;
    keyset_t t = cur; cur = nxt; nxt = t;
  }

  /* output in canonical order: sort (key, source index) records on the key */
  {
    int64_t cnt = F.found_count;
    size_t rec = (size_t)W + 1;
    uint64_t *tmp = (uint64_t *)malloc((size_t)(cnt ? cnt : 1) * rec * sizeof(uint64_t));
    R->keys = (uint64_t *)malloc((size_t)(cnt ? cnt : 1) * W * sizeof(uint64_t));
    R->flux = (int64_t *)malloc((size_t)(cnt ? cnt : 1) * n * sizeof(int64_t));
    if (!tmp || !R->keys || !R->flux) { free(tmp); rc = ORC_ENOMEM; goto done; }
    for (int64_t i = 0; i < cnt; ++i) {
      memcpy(tmp + i * rec, F.found_keys.keys + (size_t)i * W, (size_t)W * 8);
      tmp[i * rec + W] = (uint64_t)i;
    }
    g_W_cmp = W;                         /* the comparator reads the first W words */
    if (cnt > 1) qsort(tmp, (size_t)cnt, rec * sizeof(uint64_t), key_cmp);
    for (int64_t i = 0; i < cnt; ++i) {
      int64_t src = (int64_t)tmp[i * rec + W];
      memcpy(R->keys + (size_t)i * W, tmp + i * rec, (size_t)W * 8);
      memcpy(R->flux + (size_t)i * n, F.found_flux + (size_t)src * n, (size_t)n * 8);
    }
    R->count = cnt;
    free(tmp);
  }

done:
  free(cur.keys); free(nxt.keys); free(key); free(work); free(flux); free(cand); free(ra);
  free(F.found_keys.keys); free(F.found_flux);
  if (rc != ORC_OK) {
    free(R->keys); free(R->flux); free(R);
    return rc;
  }
  *out = R;
  return ORC_OK;
}

/* ------------------------------------------------------- result accessors */
int64_t orc_count(const orc_result *R) { return R->count; }
uint32_t orc_status(const orc_result *R) { return R->status; }
int orc_words(const orc_result *R) { return R->W; }
int orc_n_levels(const orc_result *R) { return R->n_levels; }
void orc_copy(const orc_result *R, uint64_t *keys, int64_t *flux) {
  if (keys) memcpy(keys, R->keys, (size_t)R->count * R->W * 8);
  if (flux) memcpy(flux, R->flux, (size_t)R->count * R->n * 8);
}
/* 6 counters per level: parents, children, unique, independent, emitted, kept */
void orc_levels(const orc_result *R, int64_t *dst) {
  for (int k = 0; k < R->n_levels; ++k) {
    const orc_level_t *L = &R->levels[k];
    int64_t *d = dst + 6 * k;
    d[0] = L->parents; d[1] = L->children; d[2] = L->unique;
    d[3] = L->independent; d[4] = L->emitted; d[5] = L->kept;
  }
}
void orc_free(orc_result *R) {
  if (!R) return;
  free(R->keys); free(R->flux); free(R);
}
