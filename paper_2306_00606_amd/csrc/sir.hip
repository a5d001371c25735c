// SIR outbreaks on the graph (Sec. 3.1) and the empirical spreading power of
// every node (Sec. 3.3), for checking Expected Force against simulated
// spreading.
//
// Model, in discrete steps: at t = 0 the index case is infected. In step t
// every node infected at the start of the step tries to infect each
// susceptible neighbour with probability beta; a susceptible node reached by
// a successful attempt is infected at t + 1, its infector being the smallest
// id among the successful attempts. Then every node infected at the start of
// the step recovers with probability mu. The outbreak ends when no node is
// infected, or at t_max.
//
// Randomness: SplitMix64's output function (Steele, Lea and Flood, 2014) of a
// counter per decision:
//   stream(r, t) = mix(mix(seed ^ r) ^ (t + 1))
//   attempt along arc e: mix(stream ^ (2 e) K), recovery of u: mix(stream ^ (2 u + 1) K)
//   index case of simulation r: high 64 bits of mix(mix(seed ^ r) ^ ~0) * n
// with K = 0xD1B54A32D192ED03; a decision of probability p succeeds when
// (value >> 11) < floor(p 2^53). Every outcome is an integer function of
// these draws, so results do not depend on scheduling.
//
// Layout: a batch of R simulations runs together, each with a byte of state,
// a candidate infector and an infector per node ([R][n] arrays). One step is
// two launches over the batch (attempts with atomicMin on the candidate,
// then infections and recoveries with one count per workgroup and
// simulation); the host reads the per-simulation counts after each step.
// After the batch, the descendants within d = 1..4 generations of the
// infection tree are summed per node over the global simulations
// (size >= n / 4, rounded up).
#include <algorithm>
#include <vector>

#include "ef_internal.h"

namespace efi {

constexpr uint64_t kSirK = 0xD1B54A32D192ED03ull;
constexpr int32_t kSirNone = 0x7FFFFFFF;

__device__ __host__ __forceinline__ uint64_t sir_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

enum : uint8_t { kSus = 0, kInf = 1, kRec = 2 };

// state S, no candidate, no infector; then the index case of each simulation
__global__ void k_sir_init(int32_t n, int32_t R, uint8_t *__restrict__ state,
                           int32_t *__restrict__ cand, int32_t *__restrict__ infector) {
  const int64_t total = (int64_t)n * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    state[i] = kSus;
    cand[i] = kSirNone;
    infector[i] = -1;
  }
}

__global__ void k_sir_seed(int32_t n, int32_t R, uint64_t seed, int64_t r0,
                           uint8_t *__restrict__ state, int32_t *__restrict__ index_out,
                           int32_t *__restrict__ active) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const uint64_t base = sir_mix(seed ^ (uint64_t)(r0 + r));
  const int32_t idx = (int32_t)__umul64hi(sir_mix(base ^ ~0ull), (uint64_t)n);
  state[(int64_t)r * n + idx] = kInf;
  index_out[r] = idx;
  active[r] = 1;
}

// attempts of step t: grid (node blocks, simulation)
__global__ __launch_bounds__(256) void k_sir_attempt(const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     int32_t n, uint64_t seed, int64_t r0,
                                                     int32_t t, uint64_t tb,
                                                     const int32_t *__restrict__ active,
                                                     const uint8_t *__restrict__ state,
                                                     int32_t *__restrict__ cand) {
  const int32_t r = blockIdx.y;
  if (active[r] == 0) return;
  const int64_t off = (int64_t)r * n;
  const uint64_t st = sir_mix(sir_mix(seed ^ (uint64_t)(r0 + r)) ^ (uint64_t)(t + 1));
  for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    if (state[off + u] != kInf) continue;
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      const int32_t w = col[e];
      if (state[off + w] != kSus) continue;
      const uint64_t x = sir_mix(st ^ ((uint64_t)(2 * (int64_t)e) * kSirK));
      if ((x >> 11) < tb) atomicMin(&cand[off + w], u);
    }
  }
}

// recoveries and infections of step t; next[r] / fresh[r] count the infected
// nodes after the step and the new infections (cleared before)
__global__ __launch_bounds__(256) void k_sir_update(int32_t n, uint64_t seed, int64_t r0,
                                                    int32_t t, uint64_t tm,
                                                    const int32_t *__restrict__ active,
                                                    uint8_t *__restrict__ state,
                                                    int32_t *__restrict__ cand,
                                                    int32_t *__restrict__ infector,
                                                    int32_t *__restrict__ next,
                                                    int32_t *__restrict__ fresh) {
  __shared__ int32_t sh[2][4];
  const int32_t r = blockIdx.y;
  if (active[r] == 0) return;
  const int64_t off = (int64_t)r * n;
  const uint64_t st = sir_mix(sir_mix(seed ^ (uint64_t)(r0 + r)) ^ (uint64_t)(t + 1));
  int32_t c_next = 0, c_new = 0;
  for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    const uint8_t s = state[off + u];
    if (s == kInf) {
      const uint64_t x = sir_mix(st ^ ((uint64_t)(2 * (int64_t)u + 1) * kSirK));
      if ((x >> 11) < tm) state[off + u] = kRec;
      else ++c_next;
    } else if (s == kSus) {
      const int32_t c = cand[off + u];
      if (c != kSirNone) {
        state[off + u] = kInf;
        infector[off + u] = c;
        cand[off + u] = kSirNone;
        ++c_next;
        ++c_new;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    c_next += __shfl_xor(c_next, o, 64);
    c_new += __shfl_xor(c_new, o, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wv] = c_next;
    sh[1][wv] = c_new;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int32_t a = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    const int32_t b = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    if (a) atomicAdd(&next[r], a);
    if (b) atomicAdd(&fresh[r], b);
  }
}

// one level of descendant counts: cur[p] += 1 + prev[c] for every infected c
// with infector p (prev null: level 1)
__global__ void k_sir_level(int32_t n, int32_t R, const int32_t *__restrict__ glob,
                            const int32_t *__restrict__ infector,
                            const int32_t *__restrict__ prev, int32_t *__restrict__ cur) {
  const int64_t total = (int64_t)n * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = (int32_t)(i / n);
    const int32_t p = infector[i];
    if (!glob[r] || p < 0) continue;
    atomicAdd(&cur[(int64_t)r * n + p], 1 + (prev ? prev[i] : 0));
  }
}

// per node: add the level-d counts of the global simulations in which it was
// infected (and, at d = 1, count those simulations)
__global__ void k_sir_accum(int32_t n, int32_t R, const int32_t *__restrict__ glob,
                            const uint8_t *__restrict__ state, const int32_t *__restrict__ cur,
                            int64_t *__restrict__ sp, int64_t *__restrict__ cnt) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    int64_t a = 0, c = 0;
    for (int32_t r = 0; r < R; ++r) {
      const int64_t i = (int64_t)r * n + v;
      if (glob[r] && state[i] != kSus) {
        a += cur[i];
        ++c;
      }
    }
    sp[v] += a;
    if (cnt) cnt[v] += c;
  }
}

__global__ void k_sir_zero(int64_t count, int32_t *__restrict__ p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_sir_zero64(int64_t count, int64_t *__restrict__ p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

static unsigned sir_blocks(int64_t threads) {
  int64_t b = (threads + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16));
}

static uint64_t sir_threshold(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return 1ull << 53;
  return (uint64_t)(p * 9007199254740992.0);
}

}  // namespace efi

using namespace efi;

extern "C" ef_status ef_sir(ef_graph *h, double beta, double mu, uint64_t seed, int32_t n_sims,
                            int32_t t_max, int32_t *index, int32_t *size, int32_t *t_end,
                            int32_t *t_peak, int64_t *sp_sum, int64_t *inf_count,
                            void *hip_stream) {
  if (!h || n_sims < 0 || t_max < 0 || !(beta >= 0.0 && beta <= 1.0) ||
      !(mu >= 0.0 && mu <= 1.0) || (n_sims > 0 && (!index || !size || !t_end || !t_peak)) ||
      !sp_sum || !inf_count) {
    set_error("ef_sir: bad arguments");
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  const int32_t n = g.n;
  if (n == 0) {
    if (n_sims > 0) {
      set_error("ef_sir: the graph has no nodes");
      return EF_ERR_ARG;
    }
    return EF_OK;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  // batch of simulations: about 1.5 GB of per-(simulation, node) state
  const int64_t per_sim = (int64_t)n * (1 + 4 + 4 + 4 + 4);
  // (and at most 32768 simulations: the simulation is the grid's y index)
  const int32_t RB = (int32_t)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)std::max(n_sims, 1), 32768,
                            (1536LL << 20) / std::max<int64_t>(per_sim, 1)}));
  const size_t bytes = (size_t)RB * (size_t)n * (1 + 4 * 4) + sizeof(int32_t) * 6 * (size_t)RB +
                       sizeof(int64_t) * 5 * (size_t)n + 4096;
  char *p = nullptr;
  ef_status s = graph_scratch(g, bytes, (void **)&p);
  if (s != EF_OK) return s;
  auto take = [&](size_t b) {
    char *q = p;
    p += (b + 255) & ~(size_t)255;
    return q;
  };
  const int64_t cells = (int64_t)RB * n;
  uint8_t *state = (uint8_t *)take((size_t)cells);
  int32_t *cand = (int32_t *)take(sizeof(int32_t) * (size_t)cells);
  int32_t *infector = (int32_t *)take(sizeof(int32_t) * (size_t)cells);
  int32_t *lvl[2] = {(int32_t *)take(sizeof(int32_t) * (size_t)cells),
                     (int32_t *)take(sizeof(int32_t) * (size_t)cells)};
  int32_t *d_index = (int32_t *)take(sizeof(int32_t) * RB);
  int32_t *d_active = (int32_t *)take(sizeof(int32_t) * RB);
  int32_t *d_cnt = (int32_t *)take(sizeof(int32_t) * 2 * RB);  // next, fresh
  int32_t *d_glob = (int32_t *)take(sizeof(int32_t) * RB);
  int64_t *d_sp = (int64_t *)take(sizeof(int64_t) * 5 * (size_t)n);  // 4 orders, then counts
  int64_t *d_ic = d_sp + 4 * (int64_t)n;
  const uint64_t tb = sir_threshold(beta), tm = sir_threshold(mu);
  const int64_t global_min = ((int64_t)n + 3) / 4;
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(k_sir_zero64, dim3(sir_blocks(5 * (int64_t)n)), dim3(256), 0, st,
                     5 * (int64_t)n, d_sp);
  std::vector<int32_t> h_cnt(2 * (size_t)RB), h_active((size_t)RB), h_glob((size_t)RB);
  const unsigned gx = sir_blocks(n);
  for (int32_t r0 = 0; r0 < n_sims && e == hipSuccess; r0 += RB) {
    const int32_t R = std::min(RB, n_sims - r0);
    hipLaunchKernelGGL(k_sir_init, dim3(sir_blocks((int64_t)R * n)), dim3(256), 0, st, n, R,
                       state, cand, infector);
    hipLaunchKernelGGL(k_sir_seed, dim3((R + 255) / 256), dim3(256), 0, st, n, R, seed,
                       (int64_t)r0, state, d_index, d_active);
    std::vector<int64_t> sz((size_t)R, 1), peak((size_t)R, 1);
    std::vector<int32_t> tpk((size_t)R, 0), tend((size_t)R, 0);
    std::fill(h_active.begin(), h_active.begin() + R, 1);
    int32_t alive = R;
    for (int32_t t = 0; t < t_max && alive > 0; ++t) {
      hipLaunchKernelGGL(k_sir_zero, dim3(1), dim3(256), 0, st, (int64_t)2 * R, d_cnt);
      hipLaunchKernelGGL(k_sir_attempt, dim3(gx, R), dim3(256), 0, st, g.row_ptr, g.col_idx, n,
                         seed, (int64_t)r0, t, tb, d_active, state, cand);
      hipLaunchKernelGGL(k_sir_update, dim3(gx, R), dim3(256), 0, st, n, seed, (int64_t)r0, t, tm,
                         d_active, state, cand, infector, d_cnt, d_cnt + R);
      e = hipMemcpyAsync(h_cnt.data(), d_cnt, sizeof(int32_t) * 2 * R, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) break;
      alive = 0;
      for (int32_t r = 0; r < R; ++r) {
        if (!h_active[r]) continue;
        const int32_t nx = h_cnt[r];
        sz[r] += h_cnt[R + r];
        tend[r] = t + 1;
        if (nx > peak[r]) {
          peak[r] = nx;
          tpk[r] = t + 1;
        }
        if (nx == 0) h_active[r] = 0;
        else ++alive;
      }
      e = hipMemcpyAsync(d_active, h_active.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) break;
    }
    if (e != hipSuccess) break;
    // outputs of the batch, and the spreading power of its global simulations
    for (int32_t r = 0; r < R; ++r) {
      size[r0 + r] = (int32_t)sz[r];
      t_end[r0 + r] = tend[r];
      t_peak[r0 + r] = tpk[r];
      h_glob[r] = sz[r] >= global_min ? 1 : 0;
    }
    e = hipMemcpyAsync(index + r0, d_index, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_glob, h_glob.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    bool any = false;
    for (int32_t r = 0; r < R; ++r) any = any || h_glob[r];
    if (any) {
      const unsigned gb = sir_blocks((int64_t)R * n);
      for (int d = 1; d <= 4; ++d) {
        int32_t *cur = lvl[d & 1], *prev = d == 1 ? nullptr : lvl[(d - 1) & 1];
        hipLaunchKernelGGL(k_sir_zero, dim3(gb), dim3(256), 0, st, (int64_t)R * n, cur);
        hipLaunchKernelGGL(k_sir_level, dim3(gb), dim3(256), 0, st, n, R, d_glob, infector, prev,
                           cur);
        hipLaunchKernelGGL(k_sir_accum, dim3(gx), dim3(256), 0, st, n, R, d_glob, state, cur,
                           d_sp + (int64_t)(d - 1) * n, d == 1 ? d_ic : nullptr);
      }
    }
    e = hipStreamSynchronize(st);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(sp_sum, d_sp, sizeof(int64_t) * 4 * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(inf_count, d_ic, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_status(e, "SIR simulations");
  return EF_OK;
}
