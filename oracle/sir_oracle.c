/*
 * CPU ORACLE for the SIR spreading-power experiment (Sylos Labini et al.,
 * "Scaling Expected Force", Sec. 3.1 model, Sec. 3.3 measured quantities).
 * TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU-baseline leg
 * call it; the GPU library never links, loads or calls it, and it shares no
 * code with that library.
 *
 * Model (Sec. 3.1), in discrete time steps t = 0, 1, 2, ...: at t = 0 the
 * index case is infected and every other node susceptible. In step t every
 * node infected at the start of the step tries to infect each susceptible
 * neighbour, independently with probability beta; a susceptible node reached
 * by at least one successful attempt is infected at t + 1, its infector being
 * the smallest id among the successful attempts (a tie-break the paper leaves
 * open). Then every node infected at the start of the step recovers with
 * probability mu. The outbreak ends when no node is infected (or at t_max).
 *
 * Randomness: every decision draws one 64-bit value from SplitMix64's output
 * function (Steele, Lea and Flood, 2014) applied to a counter:
 *   stream(r, t) = mix(mix(seed ^ r) ^ (t + 1))          simulation r, step t
 *   attempt along arc e:   mix(stream ^ ((2 e)     * 0xD1B54A32D192ED03))
 *   recovery of node u:    mix(stream ^ ((2 u + 1) * 0xD1B54A32D192ED03))
 *   index case:            high 64 bits of mix(mix(seed ^ r) ^ ~0) * n
 * and a decision with probability p succeeds when (value >> 11) <
 * floor(p * 2^53).
 *
 * Per simulation: index case, size (nodes ever infected), t_end (steps until
 * no node is infected) and t_peak (first step with the most infected nodes).
 * Over the global simulations (size >= ceil(n / 4), Sec. 3.3): for every node
 * the number of global simulations in which it was infected and, for d = 1..4,
 * the sum over them of its descendants within d generations of the infection
 * tree (the empirical spreading power of order d before averaging).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t z) { return mix(z); }

static uint64_t threshold(double p) {
  if (p <= 0.0) return 0;
  if (p >= 1.0) return 1ull << 53;
  return (uint64_t)(p * 9007199254740992.0); /* floor(p 2^53) */
}

enum { S_SUS = 0, S_INF = 1, S_REC = 2 };

int oracle_sir(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, double beta, double mu,
               uint64_t seed, int32_t n_sims, int32_t t_max, int32_t *index_out,
               int32_t *size_out, int32_t *t_end_out, int32_t *t_peak_out, int64_t *sp_sum,
               int64_t *inf_count) {
  if (n <= 0 || n_sims < 0 || t_max < 0) return 1;
  const uint64_t tb = threshold(beta), tm = threshold(mu);
  const int64_t global_min = ((int64_t)n + 3) / 4;
  uint8_t *state = (uint8_t *)malloc((size_t)n);
  int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *infector = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * 5 * (size_t)n);
  uint8_t *was_inf = (uint8_t *)malloc((size_t)n);
  if (!state || !cand || !infector || !cnt || !was_inf) return 2;
  memset(sp_sum, 0, sizeof(int64_t) * 4 * (size_t)n);
  memset(inf_count, 0, sizeof(int64_t) * (size_t)n);
  for (int32_t r = 0; r < n_sims; ++r) {
    const uint64_t base = mix(seed ^ (uint64_t)r);
    const int32_t idx =
        (int32_t)(((unsigned __int128)mix(base ^ ~0ull) * (unsigned __int128)(uint64_t)n) >> 64);
    memset(state, S_SUS, (size_t)n);
    for (int32_t v = 0; v < n; ++v) {
      cand[v] = INT32_MAX;
      infector[v] = -1;
    }
    state[idx] = S_INF;
    int64_t n_inf = 1, size = 1, peak = 1;
    int32_t t = 0, t_peak = 0;
    while (n_inf > 0 && t < t_max) {
      const uint64_t st = mix(base ^ (uint64_t)(t + 1));
      for (int32_t u = 0; u < n; ++u) {
        if (state[u] != S_INF) continue;
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
          const int32_t w = col_idx[e];
          if (state[w] != S_SUS) continue;
          const uint64_t x = mix(st ^ ((uint64_t)(2 * (int64_t)e) * 0xD1B54A32D192ED03ull));
          if ((x >> 11) < tb && u < cand[w]) cand[w] = u;
        }
      }
      /* recoveries of the nodes infected at the start of the step */
      int64_t next = 0;
      for (int32_t u = 0; u < n; ++u) {
        if (state[u] != S_INF) continue;
        const uint64_t x = mix(st ^ ((uint64_t)(2 * (int64_t)u + 1) * 0xD1B54A32D192ED03ull));
        if ((x >> 11) < tm) state[u] = S_REC;
        else ++next;
      }
      /* new infections */
      for (int32_t w = 0; w < n; ++w) {
        if (cand[w] == INT32_MAX) continue;
        state[w] = S_INF;
        infector[w] = cand[w];
        cand[w] = INT32_MAX;
        ++next;
        ++size;
      }
      ++t;
      n_inf = next;
      if (n_inf > peak) {
        peak = n_inf;
        t_peak = t;
      }
    }
    index_out[r] = idx;
    size_out[r] = (int32_t)size;
    t_end_out[r] = t;
    t_peak_out[r] = t_peak;
    if (size < global_min) continue;
    /* descendants within d generations: cnt[d][v] = sum over children c of
       (1 + cnt[d-1][c]) */
    for (int32_t v = 0; v < n; ++v) {
      was_inf[v] = state[v] != S_SUS;
      cnt[v] = 0;
    }
    for (int d = 1; d <= 4; ++d) {
      int32_t *cur = cnt + (size_t)d * n, *prev = cnt + (size_t)(d - 1) * n;
      for (int32_t v = 0; v < n; ++v) cur[v] = 0;
      for (int32_t c = 0; c < n; ++c)
        if (infector[c] >= 0) cur[infector[c]] += 1 + prev[c];
      for (int32_t v = 0; v < n; ++v)
        if (was_inf[v]) sp_sum[(size_t)(d - 1) * n + v] += cur[v];
    }
    for (int32_t v = 0; v < n; ++v)
      if (was_inf[v]) inf_count[v] += 1;
  }
  free(state);
  free(cand);
  free(infector);
  free(cnt);
  free(was_inf);
  return 0;
}
