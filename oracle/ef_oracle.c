/*
 * CPU ORACLE for the Expected Force (EF) of every node of a simple undirected
 * graph. TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
 * benchmark's CPU-baseline leg call it; the GPU library never links, loads or
 * calls it, and it shares no code with that library.
 *
 * What it computes (Sylos Labini et al., "Scaling Expected Force", Sec. 3.3,
 * Eq. 1, with the cluster multiplicities of Algorithm 1):
 *
 *   For a seed s, list every ordered pair of transmission events that starts
 *   from the infected set {s}:
 *     event 1:  s infects a neighbour y of s;
 *     event 2:  an infected node x in {s, y} infects a neighbour z of x that
 *               is still susceptible (z not in {s, y}).
 *   Each sequence ends in the infected cluster J = {s, y, z}. Its degree d_J
 *   is the number of edges with exactly one endpoint in J (Fig. 1 caption),
 *   i.e. (sum of the degrees of the three nodes) - 2 * (edges inside J).
 *   H_s(d) counts the sequences whose cluster has degree d. A star y-s-z is
 *   reached by two event orders and a path s-y-z by one, which are the +2 /
 *   +1 / +1 credits of Algorithm 1 (Phase 2); a triangle's node set is
 *   reached four times from each of its nodes.
 *
 *   N_s = sum_d H_s(d),  D_s = sum_d d * H_s(d)   (exact integers)
 *   EF_s = - sum_c (d_c / D_s) log(d_c / D_s)      (Eq. 1, natural log)
 *        = sum_{d > 0} H_s(d) * (d / D_s) * log1p((D_s - d) / d)
 *   with EF_s = +0.0 when D_s = 0 or N_s <= 1, and 0 log 0 taken as 0.
 *
 * Every term of the last sum is non-negative, so it is evaluated without
 * cancellation: the distinct degrees are visited in ascending order and the
 * terms summed with Neumaier's compensated summation in double precision.
 *
 * The three adjacency tests inside J are done one by one: membership in N(s)
 * is read from a flag array stamped for the current seed, membership in N(y)
 * from a second array stamped for the current (s, y).
 *
 * The seed loop may run on several OpenMP threads (dynamic schedule, chunk 2,
 * as in the paper's vertex-centric CPU version, Sec. 4.1); each seed is still
 * computed by one thread in the order above, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_ERR_ARG 1
#define ORACLE_ERR_NOMEM 2

typedef struct {
  int64_t *hist;    /* hist[d] = H_s(d), length max_d + 1 */
  int32_t *touched; /* distinct d values seen for the current seed */
  int32_t n_touched;
  int64_t *mark_s;  /* mark_s[x] == stamp  <=>  x in N(s) */
  int64_t *mark_y;  /* mark_y[x] == stamp2 <=>  x in N(y) */
} scratch_t;

static int scratch_init(scratch_t *w, int32_t n, int64_t max_d) {
  memset(w, 0, sizeof(*w));
  w->hist = (int64_t *)calloc((size_t)max_d + 1, sizeof(int64_t));
  w->touched = (int32_t *)malloc(sizeof(int32_t) * ((size_t)max_d + 1));
  w->mark_s = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  w->mark_y = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!w->hist || !w->touched || !w->mark_s || !w->mark_y) return ORACLE_ERR_NOMEM;
  for (int32_t i = 0; i <= n; ++i) w->mark_s[i] = w->mark_y[i] = -1;
  return ORACLE_OK;
}

static void scratch_free(scratch_t *w) {
  free(w->hist);
  free(w->touched);
  free(w->mark_s);
  free(w->mark_y);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static inline void hist_add(scratch_t *w, int64_t d) {
  if (w->hist[d] == 0) w->touched[w->n_touched++] = (int32_t)d;
  w->hist[d] += 1;
}

/* Enumerate the event sequences of seed s into w->hist. */
static void seed_histogram(int32_t s, const int32_t *row_ptr, const int32_t *col_idx,
                           scratch_t *w, int64_t *stamp2) {
  const int32_t s0 = row_ptr[s], s1 = row_ptr[s + 1];
  const int64_t ks = s1 - s0;
  for (int32_t e = s0; e < s1; ++e) w->mark_s[col_idx[e]] = s;
  for (int32_t e1 = s0; e1 < s1; ++e1) {
    const int32_t y = col_idx[e1]; /* event 1: s -> y */
    const int32_t y0 = row_ptr[y], y1 = row_ptr[y + 1];
    const int64_t ky = y1 - y0;
    const int64_t st = (*stamp2)++;
    for (int32_t e = y0; e < y1; ++e) w->mark_y[col_idx[e]] = st;
    /* event 2 by s: s -> z, z in N(s) \ {s, y} */
    for (int32_t e2 = s0; e2 < s1; ++e2) {
      const int32_t z = col_idx[e2];
      if (z == y || z == s) continue;
      const int64_t kz = row_ptr[z + 1] - row_ptr[z];
      const int64_t internal = 1 /* s~y */ + 1 /* s~z */ + (w->mark_y[z] == st ? 1 : 0);
      hist_add(w, ks + ky + kz - 2 * internal);
    }
    /* event 2 by y: y -> z, z in N(y) \ {s, y} */
    for (int32_t e2 = y0; e2 < y1; ++e2) {
      const int32_t z = col_idx[e2];
      if (z == s || z == y) continue;
      const int64_t kz = row_ptr[z + 1] - row_ptr[z];
      const int64_t internal = 1 /* s~y */ + 1 /* y~z */ + (w->mark_s[z] == s ? 1 : 0);
      hist_add(w, ks + ky + kz - 2 * internal);
    }
  }
}

/* N, D and EF from the histogram; clears the histogram. */
static void seed_finish(scratch_t *w, int64_t *N_out, int64_t *D_out, double *EF_out) {
  qsort(w->touched, (size_t)w->n_touched, sizeof(int32_t), cmp_i32);
  int64_t N = 0, D = 0;
  for (int32_t t = 0; t < w->n_touched; ++t) {
    const int64_t d = w->touched[t];
    N += w->hist[d];
    D += d * w->hist[d];
  }
  double ef = 0.0;
  if (D > 0 && N > 1) {
    double sum = 0.0, comp = 0.0; /* Neumaier */
    const double Dd = (double)D;
    for (int32_t t = 0; t < w->n_touched; ++t) {
      const int64_t d = w->touched[t];
      if (d == 0) continue; /* 0 log 0 = 0 */
      const double term =
          (double)w->hist[d] * ((double)d / Dd) * log1p((double)(D - d) / (double)d);
      const double nt = sum + term;
      if (fabs(sum) >= fabs(term)) comp += (sum - nt) + term;
      else comp += (term - nt) + sum;
      sum = nt;
    }
    ef = sum + comp;
    if (ef <= 0.0) ef = 0.0; /* never -0.0 */
  }
  for (int32_t t = 0; t < w->n_touched; ++t) w->hist[w->touched[t]] = 0;
  w->n_touched = 0;
  *N_out = N;
  *D_out = D;
  *EF_out = ef;
}

static int32_t max_degree(int32_t n, const int32_t *row_ptr) {
  int32_t m = 0;
  for (int32_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] - row_ptr[i] > m) m = row_ptr[i + 1] - row_ptr[i];
  return m;
}

/*
 * Expected Force with j = 3 transmission events (Sec. 3.3 defines EF for a
 * number j of events and uses j = 2; the sequences are counted the same way
 * as for j = 2, one per ordered list of events):
 *     event 1:  s infects a neighbour y of s;
 *     event 2:  x2 in {s, y} infects a susceptible neighbour z of x2;
 *     event 3:  x3 in {s, y, z} infects a susceptible neighbour w of x3.
 * The cluster is J = {s, y, z, w}; its degree is the number of edges with
 * exactly one endpoint in J, (sum of the four degrees) - 2 * (edges inside J),
 * the internal edges found by the membership tests below. H_s, N_s, D_s and
 * EF_s then follow exactly as for j = 2 (seed_finish).
 */
static void seed_histogram3(int32_t s, const int32_t *row_ptr, const int32_t *col_idx,
                            scratch_t *w, int64_t *mark_z, int64_t *stamp2, int64_t *stamp3) {
  const int32_t s0 = row_ptr[s], s1 = row_ptr[s + 1];
  const int64_t ks = s1 - s0;
  for (int32_t e = s0; e < s1; ++e) w->mark_s[col_idx[e]] = s;
  for (int32_t e1 = s0; e1 < s1; ++e1) {
    const int32_t y = col_idx[e1]; /* event 1: s -> y */
    const int32_t y0 = row_ptr[y], y1 = row_ptr[y + 1];
    const int64_t ky = y1 - y0;
    const int64_t st = (*stamp2)++;
    for (int32_t e = y0; e < y1; ++e) w->mark_y[col_idx[e]] = st;
    /* event 2: x2 -> z, from s (pass 0) or from y (pass 1) */
    for (int pass = 0; pass < 2; ++pass) {
      const int32_t x2 = pass == 0 ? s : y;
      for (int32_t e2 = row_ptr[x2]; e2 < row_ptr[x2 + 1]; ++e2) {
        const int32_t z = col_idx[e2];
        const int z_infected = z == s || z == y; /* z must be susceptible */
        if (z_infected) continue;
        const int32_t z0 = row_ptr[z], z1 = row_ptr[z + 1];
        const int64_t kz = z1 - z0;
        const int64_t st3 = (*stamp3)++;
        for (int32_t e = z0; e < z1; ++e) mark_z[col_idx[e]] = st3;
        /* edges inside {s, y, z}: s~y, and z's edges to s and to y */
        const int64_t in3 = 1 + (w->mark_s[z] == s ? 1 : 0) + (w->mark_y[z] == st ? 1 : 0);
        /* event 3: x3 -> v, x3 in {s, y, z}, v not in {s, y, z} */
        const int32_t tri[3] = {s, y, z};
        for (int t = 0; t < 3; ++t) {
          const int32_t x3 = tri[t];
          for (int32_t e3 = row_ptr[x3]; e3 < row_ptr[x3 + 1]; ++e3) {
            const int32_t v = col_idx[e3];
            if (v == s || v == y || v == z) continue;
            const int64_t kv = row_ptr[v + 1] - row_ptr[v];
            const int64_t cv = (w->mark_s[v] == s ? 1 : 0) + (w->mark_y[v] == st ? 1 : 0) +
                               (mark_z[v] == st3 ? 1 : 0);
            hist_add(w, ks + ky + kz + kv - 2 * (in3 + cv));
          }
        }
      }
    }
  }
}

/* EF with j = 3 events for `seeds` (all nodes when NULL); as oracle_ef. */
int oracle_ef3(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
               const int32_t *seeds, int32_t n_seeds, int64_t *N_out, int64_t *D_out,
               double *EF_out, int32_t n_threads) {
  if (n < 0 || !row_ptr || (n > 0 && row_ptr[n] > 0 && !col_idx)) return ORACLE_ERR_ARG;
  const int32_t count = seeds ? n_seeds : n;
  if (count < 0) return ORACLE_ERR_ARG;
  if (count == 0) return ORACLE_OK;
  for (int32_t t = 0; seeds && t < count; ++t)
    if (seeds[t] < 0 || seeds[t] >= n) return ORACLE_ERR_ARG;
  const int64_t max_d = 4 * (int64_t)max_degree(n, row_ptr);
  int status = ORACLE_OK;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
#pragma omp parallel
  {
    scratch_t w;
    int64_t *mark_z = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int ok = scratch_init(&w, n, max_d) == ORACLE_OK && mark_z;
    if (!ok) {
#pragma omp atomic write
      status = ORACLE_ERR_NOMEM;
    } else {
      for (int32_t i = 0; i <= n; ++i) mark_z[i] = -1;
    }
    int64_t stamp2 = 0, stamp3 = 0;
#pragma omp for schedule(dynamic, 2)
    for (int32_t t = 0; t < count; ++t) {
      if (!ok) continue;
      const int32_t s = seeds ? seeds[t] : t;
      seed_histogram3(s, row_ptr, col_idx, &w, mark_z, &stamp2, &stamp3);
      seed_finish(&w, &N_out[t], &D_out[t], &EF_out[t]);
    }
    scratch_free(&w);
    free(mark_z);
  }
  return status;
}

/* H_s for j = 3 events, as oracle_histogram. */
int64_t oracle_histogram3(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          int32_t s, int64_t *deg_out, int64_t *count_out, int64_t cap) {
  if (n <= 0 || s < 0 || s >= n || !row_ptr) return -1;
  scratch_t w;
  int64_t *mark_z = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!mark_z || scratch_init(&w, n, 4 * (int64_t)max_degree(n, row_ptr)) != ORACLE_OK) {
    scratch_free(&w);
    free(mark_z);
    return -1;
  }
  for (int32_t i = 0; i <= n; ++i) mark_z[i] = -1;
  int64_t stamp2 = 0, stamp3 = 0;
  seed_histogram3(s, row_ptr, col_idx, &w, mark_z, &stamp2, &stamp3);
  qsort(w.touched, (size_t)w.n_touched, sizeof(int32_t), cmp_i32);
  const int64_t m = w.n_touched;
  for (int64_t t = 0; t < m && t < cap; ++t) {
    deg_out[t] = w.touched[t];
    count_out[t] = w.hist[w.touched[t]];
  }
  scratch_free(&w);
  free(mark_z);
  return m;
}

/*
 * EF of the seeds `seeds[0..n_seeds)` (all nodes 0..n-1 when seeds == NULL,
 * then n_seeds is ignored). Outputs are position-aligned with the seed list.
 * The CSR must describe a simple undirected graph with sorted rows; it is not
 * validated here. n_threads <= 0 uses the OpenMP default.
 */
int oracle_ef(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
              const int32_t *seeds, int32_t n_seeds, int64_t *N_out, int64_t *D_out,
              double *EF_out, int32_t n_threads) {
  if (n < 0 || !row_ptr || (n > 0 && row_ptr[n] > 0 && !col_idx)) return ORACLE_ERR_ARG;
  const int32_t count = seeds ? n_seeds : n;
  if (count < 0) return ORACLE_ERR_ARG;
  if (count == 0) return ORACLE_OK;
  for (int32_t t = 0; seeds && t < count; ++t)
    if (seeds[t] < 0 || seeds[t] >= n) return ORACLE_ERR_ARG;
  const int64_t max_d = 3 * (int64_t)max_degree(n, row_ptr);
  int status = ORACLE_OK;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
#pragma omp parallel
  {
    scratch_t w;
    int ok = scratch_init(&w, n, max_d) == ORACLE_OK;
    if (!ok) {
#pragma omp atomic write
      status = ORACLE_ERR_NOMEM;
    }
    int64_t stamp2 = 0;
#pragma omp for schedule(dynamic, 2)
    for (int32_t t = 0; t < count; ++t) {
      if (!ok) continue;
      const int32_t s = seeds ? seeds[t] : t;
      seed_histogram(s, row_ptr, col_idx, &w, &stamp2);
      seed_finish(&w, &N_out[t], &D_out[t], &EF_out[t]);
    }
    scratch_free(&w);
  }
  return status;
}

/*
 * The histogram H_s itself for one seed: writes up to `cap` (degree, count)
 * pairs in ascending degree order and returns the number of distinct degrees
 * (which may exceed cap), or -1 on bad arguments / allocation failure.
 */
int64_t oracle_histogram(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                         int32_t s, int64_t *deg_out, int64_t *count_out, int64_t cap) {
  if (n <= 0 || s < 0 || s >= n || !row_ptr) return -1;
  scratch_t w;
  if (scratch_init(&w, n, 3 * (int64_t)max_degree(n, row_ptr)) != ORACLE_OK) {
    scratch_free(&w);
    return -1;
  }
  int64_t stamp2 = 0;
  seed_histogram(s, row_ptr, col_idx, &w, &stamp2);
  qsort(w.touched, (size_t)w.n_touched, sizeof(int32_t), cmp_i32);
  const int64_t m = w.n_touched;
  for (int64_t t = 0; t < m && t < cap; ++t) {
    deg_out[t] = w.touched[t];
    count_out[t] = w.hist[w.touched[t]];
  }
  scratch_free(&w);
  return m;
}
