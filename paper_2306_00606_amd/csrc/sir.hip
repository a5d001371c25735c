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
// Layout: a batch of R simulations runs together. Per (simulation, node): a
// state byte and a candidate word, which holds the smallest successful
// attempter while the node is susceptible and keeps it as the infector once
// the node is infected; per simulation two frontier lists of length n (the
// infected nodes at the start of a step, and the next step's list). One step
// is four launches: a one-workgroup prefix over the simulations' frontier
// lengths, the attempts (one flat index space over all frontiers, each
// wavefront expanding the arcs of 64 frontier nodes with a wave-wide prefix of
// their degrees), a prefix over frontier + new infections, and the update
// (new infections become infected, frontier nodes recover or stay). Lists
// grow with wave-aggregated atomic appends; the order of entries varies from
// run to run but no outcome depends on it. Per-simulation counters stay on
// the device; the host checks every few steps whether any outbreak is alive.
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

constexpr int32_t kSirMaxBatch = 1024;  // simulations per batch: one prefix workgroup
constexpr int32_t kSirCheck = 8;        // steps between the host's checks for live outbreaks
constexpr unsigned kSirGrid = 2048;     // workgroups of the frontier kernels (grid-stride)

constexpr int32_t kSirPad = 32;  // int32 stride of the append counters: one 128-byte line each
constexpr int32_t kSirTab = kSirMaxBatch + 1;  // stride of the per-batch tables below

// per simulation of a batch
struct SirSim {
  int32_t F;      // frontier length: infected nodes at the start of the step
  int32_t fresh;  // new infections of the step (set between attempts and update)
  int32_t size, peak, t_peak, t_end, index, pad;
  int64_t fsteps;  // frontier nodes summed over the steps run
};

// exclusive prefix over one value per thread of a 1024-thread workgroup
__device__ int32_t sir_scan1024(int32_t v, int32_t *sh, int32_t *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) sh[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int w = 0; w < 16; ++w) {
      const int32_t x = sh[w];
      sh[w] = run;
      run += x;
    }
    sh[16] = run;
  }
  __syncthreads();
  *total = sh[16];
  return sh[wv] + incl - v;
}

// state S and no candidate everywhere
__global__ void k_sir_init(int32_t n, int32_t R, uint8_t *__restrict__ state,
                           int32_t *__restrict__ cand) {
  const int64_t total = (int64_t)n * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    state[i] = kSus;
    cand[i] = kSirNone;
  }
}

// index case of each simulation: infected, alone in the frontier
__global__ void k_sir_seed(int32_t n, int32_t R, uint64_t seed, int64_t r0,
                           uint8_t *__restrict__ state, int32_t *__restrict__ cur,
                           SirSim *__restrict__ sims, int32_t *__restrict__ nxc) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const uint64_t base = sir_mix(seed ^ (uint64_t)(r0 + r));
  const int32_t idx = (int32_t)__umul64hi(sir_mix(base ^ ~0ull), (uint64_t)n);
  state[(int64_t)r * n + idx] = kInf;
  cur[(int64_t)r * n] = idx;
  SirSim s;
  s.F = 1;
  s.fresh = 0;
  s.size = 1;
  s.peak = 1;
  s.t_peak = 0;
  s.t_end = 0;
  s.index = idx;
  s.pad = 0;
  s.fsteps = 0;
  sims[r] = s;
  nxc[(int64_t)r * kSirPad] = 0;
}

// Start of step t: fold step t - 1 into each simulation's outcome (the next
// frontier becomes the frontier), then the attempts' table: prefix over the
// frontier lengths in units of 64 nodes (tab[0..R]) and the lengths
// (tab[kSirTab + a]); and the number of live simulations.
__global__ __launch_bounds__(1024) void k_sir_prep(int32_t R, int32_t t, SirSim *__restrict__ sims,
                                                   int32_t *__restrict__ nxc,
                                                   int32_t *__restrict__ tab,
                                                   int32_t *__restrict__ alive) {
  __shared__ int32_t sh[17];
  const int32_t a = threadIdx.x;
  int32_t len = 0, act = 0;
  if (a < R) {
    SirSim s = sims[a];
    if (t > 0 && s.F > 0) {
      const int32_t nx = nxc[(int64_t)a * kSirPad];
      s.fsteps += s.F;
      s.size += s.fresh;
      s.t_end = t;
      if (nx > s.peak) {
        s.peak = nx;
        s.t_peak = t;
      }
      s.F = nx;
    }
    s.fresh = 0;
    sims[a] = s;
    nxc[(int64_t)a * kSirPad] = 0;
    tab[kSirTab + a] = s.F;
    len = (s.F + 63) >> 6;
    act = s.F > 0 ? 1 : 0;
  }
  int32_t tot;
  const int32_t ex = sir_scan1024(len, sh, &tot);
  if (a < R) tab[a] = ex;
  if (a == 0) tab[R] = tot;
  __syncthreads();
  int32_t na;
  sir_scan1024(act, sh, &na);
  if (a == 0) *alive = na;
}

// Between attempts and update: the entries appended so far are the step's
// new infections. The update's table: prefix over frontier + new lengths in
// units of 256 entries (tab[0..R]), the frontier lengths (tab[kSirTab + a])
// and the new counts (tab[2 kSirTab + a]).
__global__ __launch_bounds__(1024) void k_sir_prep_u(int32_t R, SirSim *__restrict__ sims,
                                                     const int32_t *__restrict__ nxc,
                                                     int32_t *__restrict__ tab) {
  __shared__ int32_t sh[17];
  const int32_t a = threadIdx.x;
  int32_t len = 0;
  if (a < R) {
    const int32_t F = sims[a].F, fr = nxc[(int64_t)a * kSirPad];
    sims[a].fresh = fr;
    tab[kSirTab + a] = F;
    tab[2 * kSirTab + a] = fr;
    len = F > 0 ? (F + fr + 255) >> 8 : 0;
  }
  int32_t tot;
  const int32_t ex = sir_scan1024(len, sh, &tot);
  if (a < R) tab[a] = ex;
  if (a == 0) tab[R] = tot;
}

// the simulation whose range of work units holds unit c: the largest a with
// p[a] <= c (p[0] = 0 <= c < p[R])
__device__ __forceinline__ int32_t sir_owner(const int32_t *p, int32_t R, int32_t c) {
  int32_t lo = 0, hi = R;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (p[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

// orders this wavefront's LDS accesses (written by one lane, read by another)
__device__ __forceinline__ void sir_wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Appends to a simulation's next frontier, gathered per wavefront in LDS and
// written with one atomic reservation per flush (not one per 64 entries:
// every wavefront of a simulation reserves on the same counter).
constexpr int32_t kSirBuf = 256;

struct SirBuf {
  int32_t *lds;  // this wavefront's kSirBuf entries
  int32_t cnt;   // entries held (the same in every lane)
  int32_t sim;   // simulation slot they belong to (-1: none)
};

__device__ __forceinline__ void sir_flush(SirBuf &b, int32_t *__restrict__ nxc,
                                          int32_t *__restrict__ lists, int32_t n) {
  if (b.cnt > 0) {
    const int lane = threadIdx.x & 63;
    sir_wave_fence();
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(&nxc[(int64_t)b.sim * kSirPad], b.cnt);
    base = __shfl(base, 0, 64);
    int32_t *dst = lists + (int64_t)b.sim * n + base;
    for (int32_t i = lane; i < b.cnt; i += 64) dst[i] = b.lds[i];
    sir_wave_fence();
  }
  b.cnt = 0;
}

// the wavefront moves on to simulation a: flush what belongs to another one
__device__ __forceinline__ void sir_switch(SirBuf &b, int32_t a, int32_t *__restrict__ nxc,
                                           int32_t *__restrict__ lists, int32_t n) {
  if (b.sim != a) {
    sir_flush(b, nxc, lists, n);
    b.sim = a;
  }
}

__device__ __forceinline__ void sir_push(SirBuf &b, bool take, int32_t v,
                                         int32_t *__restrict__ nxc, int32_t *__restrict__ lists,
                                         int32_t n) {
  const unsigned long long m = __ballot(take);
  if (m == 0) return;
  const int32_t k = __popcll(m);
  if (b.cnt + k > kSirBuf) sir_flush(b, nxc, lists, n);
  const int lane = threadIdx.x & 63;
  if (take) b.lds[b.cnt + __popcll(m & ((1ull << lane) - 1))] = v;
  b.cnt += k;
}

// Attempts of step t along every arc of every frontier node. A wavefront
// takes 64 frontier nodes of one simulation and walks their arcs 256 at a
// time (four per lane, so that the loads and atomics of the four overlap),
// the owner of each arc found by a search over the wave-wide degree prefix.
__global__ __launch_bounds__(256) void k_sir_attempt(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col, int32_t n, uint64_t seed,
    int64_t r0, int32_t t, uint64_t tb, int32_t R, const int32_t *__restrict__ tab,
    int32_t *__restrict__ nxc, const int32_t *__restrict__ cur, const uint8_t *__restrict__ state,
    int32_t *__restrict__ cand, int32_t *__restrict__ nxt, int64_t *__restrict__ wk) {
  __shared__ int32_t sp[kSirTab], sF[kSirMaxBatch];
  __shared__ int32_t sbuf[4][kSirBuf];
  __shared__ int32_t shw[4][256], shu[4][256];  // successful attempts: target, attempter
  for (int32_t x = threadIdx.x; x <= R; x += blockDim.x) sp[x] = tab[x];
  for (int32_t x = threadIdx.x; x < R; x += blockDim.x) sF[x] = tab[kSirTab + x];
  __syncthreads();
  const int32_t chunks = sp[R];
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1;
  const int32_t nw = (int32_t)gridDim.x * 4;
  SirBuf buf{sbuf[threadIdx.x >> 6], 0, -1};
  int32_t *hw = shw[threadIdx.x >> 6], *hu = shu[threadIdx.x >> 6];
  int64_t arcs = 0;  // arcs walked by this wavefront (work count)
  for (int32_t c = (int32_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < chunks; c += nw) {
    const int32_t a = sir_owner(sp, R, c);
    sir_switch(buf, a, nxc, nxt, n);
    const int64_t off = (int64_t)a * n;
    const int32_t i = (c - sp[a]) * 64 + lane;
    int32_t u = 0, beg = 0, deg = 0;
    if (i < sF[a]) {
      u = cur[off + i];
      beg = row_ptr[u];
      deg = row_ptr[u + 1] - beg;
    }
    int32_t incl = deg;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const int32_t tot = __shfl(incl, 63, 64), excl = incl - deg;
    arcs += tot;
    const uint64_t st = sir_mix(sir_mix(seed ^ (uint64_t)(r0 + a)) ^ (uint64_t)(t + 1));
    for (int32_t jb = 0; jb < tot; jb += 256) {
      int32_t e[4], ou[4], w[4];
      bool hit[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t j = jb + 64 * q + lane;
        // owner lane of arc j: the largest k with excl[k] <= j
        int32_t k = 0;
        for (int32_t sstep = 32; sstep > 0; sstep >>= 1) {
          const int32_t ex = __shfl(excl, k + sstep, 64);
          if (ex <= j) k += sstep;
        }
        const int32_t ob = __shfl(beg, k, 64), oe = __shfl(excl, k, 64);
        ou[q] = __shfl(u, k, 64);
        e[q] = ob + (j - oe);
        // the draw depends on the arc alone: only a successful one needs the
        // target and its state
        const uint64_t x = sir_mix(st ^ ((uint64_t)(2 * (int64_t)e[q]) * kSirK));
        hit[q] = j < tot && (x >> 11) < tb;
      }
      // lanes without a success read arc 0 and its target (valid: tot > 0)
#pragma unroll
      for (int q = 0; q < 4; ++q) w[q] = col[hit[q] ? e[q] : 0];
#pragma unroll
      for (int q = 0; q < 4; ++q) hit[q] = hit[q] & (state[off + w[q]] == kSus);
      // gather the successes, so that their atomics go out together
      int32_t nh = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const unsigned long long m = __ballot(hit[q]);
        if (hit[q]) {
          const int32_t r = nh + __popcll(m & below);
          hw[r] = w[q];
          hu[r] = ou[q];
        }
        nh += __popcll(m);
      }
      sir_wave_fence();
      for (int32_t r = 0; r < nh; r += 64) {
        bool fresh = false;
        int32_t x = 0;
        if (r + lane < nh) {
          x = hw[r + lane];
          fresh = atomicMin(&cand[off + x], hu[r + lane]) == kSirNone;
        }
        sir_push(buf, fresh, x, nxc, nxt, n);
      }
      sir_wave_fence();
    }
  }
  sir_flush(buf, nxc, nxt, n);
  // each wavefront owns one slot of the arc counts: no atomic needed
  if (lane == 0) wk[blockIdx.x * 4 + (threadIdx.x >> 6)] += arcs;
}

// Update of step t, 256 entries per wavefront (four per lane): the step's new
// infections become infected; frontier nodes recover with probability mu or
// stay in the next frontier.
__global__ __launch_bounds__(256) void k_sir_update(int32_t n, uint64_t seed, int64_t r0,
                                                    int32_t t, uint64_t tm, int32_t R,
                                                    const int32_t *__restrict__ tab,
                                                    int32_t *__restrict__ nxc,
                                                    const int32_t *__restrict__ cur,
                                                    uint8_t *__restrict__ state,
                                                    int32_t *__restrict__ nxt) {
  __shared__ int32_t sp[kSirTab], sF[kSirMaxBatch], sfr[kSirMaxBatch];
  __shared__ int32_t sbuf[4][kSirBuf];
  for (int32_t x = threadIdx.x; x <= R; x += blockDim.x) sp[x] = tab[x];
  for (int32_t x = threadIdx.x; x < R; x += blockDim.x) {
    sF[x] = tab[kSirTab + x];
    sfr[x] = tab[2 * kSirTab + x];
  }
  __syncthreads();
  const int32_t units = sp[R];
  const int lane = threadIdx.x & 63;
  const int32_t nw = (int32_t)gridDim.x * 4;
  SirBuf buf{sbuf[threadIdx.x >> 6], 0, -1};
  for (int32_t c = (int32_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < units; c += nw) {
    const int32_t a = sir_owner(sp, R, c);
    sir_switch(buf, a, nxc, nxt, n);
    const int32_t F = sF[a], fr = sfr[a];
    const int64_t off = (int64_t)a * n;
    const int32_t i0 = (c - sp[a]) * 256 + lane;
    const uint64_t st = sir_mix(sir_mix(seed ^ (uint64_t)(r0 + a)) ^ (uint64_t)(t + 1));
    int32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t i = i0 + 64 * q;
      // entries [0, fr) of the next list are the new infections; then the
      // frontier (lanes past the end read frontier entry 0)
      const int32_t *src = i < fr ? nxt + off + i : cur + off + (i < fr + F ? i - fr : 0);
      v[q] = *src;
    }
    bool keep[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t i = i0 + 64 * q;
      keep[q] = false;
      if (i < fr) {
        state[off + v[q]] = kInf;
      } else if (i < fr + F) {
        const uint64_t x = sir_mix(st ^ ((uint64_t)(2 * (int64_t)v[q] + 1) * kSirK));
        if ((x >> 11) < tm) state[off + v[q]] = kRec;
        else keep[q] = true;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) sir_push(buf, keep[q], v[q], nxc, nxt, n);
  }
  sir_flush(buf, nxc, nxt, n);
}

// one level of descendant counts over the global simulations (slots gl[]):
// cur[p] += 1 + prev[c] for every infected c with infector p (prev null:
// level 1); grid (node blocks, global simulation)
__global__ void k_sir_level(int32_t n, const int32_t *__restrict__ gl,
                            const uint8_t *__restrict__ state, const int32_t *__restrict__ cand,
                            const int32_t *__restrict__ prev, int32_t *__restrict__ cur) {
  const int64_t off = (int64_t)gl[blockIdx.y] * n;
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    if (state[off + v] == kSus) continue;
    const int32_t p = cand[off + v];
    if (p == kSirNone) continue;  // the index case
    atomicAdd(&cur[off + p], 1 + (prev ? prev[off + v] : 0));
  }
}

// per node: add the level-d counts of the G global simulations in which it was
// infected (and, at d = 1, count those simulations)
__global__ void k_sir_accum(int32_t n, int32_t G, const int32_t *__restrict__ gl,
                            const uint8_t *__restrict__ state, const int32_t *__restrict__ cur,
                            int64_t *__restrict__ sp, int64_t *__restrict__ cnt) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    int64_t a = 0, c = 0;
    for (int32_t j = 0; j < G; ++j) {
      const int64_t i = (int64_t)gl[j] * n + v;
      if (state[i] != kSus) {
        a += cur[i];
        ++c;
      }
    }
    sp[v] += a;
    if (cnt) cnt[v] += c;
  }
}

// zero the rows of the global simulations; grid (node blocks, global simulation)
__global__ void k_sir_zero_rows(int32_t n, const int32_t *__restrict__ gl,
                                int32_t *__restrict__ p) {
  const int64_t off = (int64_t)gl[blockIdx.y] * n;
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    p[off + v] = 0;
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
                            int64_t *work, double *phase_ms, void *hip_stream) {
  if (!h || n_sims < 0 || t_max < 0 || !(beta >= 0.0 && beta <= 1.0) ||
      !(mu >= 0.0 && mu <= 1.0) || (n_sims > 0 && (!index || !size || !t_end || !t_peak)) ||
      !sp_sum || !inf_count) {
    set_error("ef_sir: bad arguments");
    return EF_ERR_ARG;
  }
  if (work) work[0] = work[1] = 0;
  if (phase_ms) phase_ms[0] = phase_ms[1] = phase_ms[2] = 0.0;
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
  // batch: about 3 GB of per-(simulation, node) state (13 bytes), at most
  // one prefix workgroup of simulations
  const int64_t per_sim = (int64_t)n * (1 + 4 + 4 + 4);
  const int32_t RB = (int32_t)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)std::max(n_sims, 1), (int64_t)kSirMaxBatch,
                            (3LL << 30) / std::max<int64_t>(per_sim, 1)}));
  const size_t cells = (size_t)RB * (size_t)n;
  const size_t bytes = cells * 13 + sizeof(SirSim) * RB + sizeof(int32_t) * kSirPad * RB +
                       sizeof(int32_t) * (5 * (size_t)kSirTab + RB + 1) +
                       sizeof(int64_t) * (5 * (size_t)n + kSirGrid * 4) + 16 * 256;
  char *p = nullptr;
  ef_status s = graph_scratch(g, bytes, (void **)&p);
  if (s != EF_OK) return s;
  auto take = [&](size_t b) {
    char *q = p;
    p += (b + 255) & ~(size_t)255;
    return q;
  };
  uint8_t *state = (uint8_t *)take(cells);
  int32_t *cand = (int32_t *)take(sizeof(int32_t) * cells);
  int32_t *list[2] = {(int32_t *)take(sizeof(int32_t) * cells),
                      (int32_t *)take(sizeof(int32_t) * cells)};
  SirSim *d_sims = (SirSim *)take(sizeof(SirSim) * RB);
  int32_t *d_nxc = (int32_t *)take(sizeof(int32_t) * kSirPad * RB);
  int32_t *d_tabA = (int32_t *)take(sizeof(int32_t) * 2 * kSirTab);
  int32_t *d_tabU = (int32_t *)take(sizeof(int32_t) * 3 * kSirTab);
  int32_t *d_glob = (int32_t *)take(sizeof(int32_t) * RB + sizeof(int32_t));
  int32_t *d_alive = d_glob + RB;
  int64_t *d_sp = (int64_t *)take(sizeof(int64_t) * 5 * (size_t)n);  // 4 orders, then counts
  int64_t *d_ic = d_sp + 4 * (int64_t)n;
  int64_t *d_wk = (int64_t *)take(sizeof(int64_t) * kSirGrid * 4);  // arcs per attempt wavefront
  const uint64_t tb = sir_threshold(beta), tm = sir_threshold(mu);
  const int64_t global_min = ((int64_t)n + 3) / 4;
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(k_sir_zero64, dim3(sir_blocks(5 * (int64_t)n)), dim3(256), 0, st,
                     5 * (int64_t)n, d_sp);
  hipLaunchKernelGGL(k_sir_zero64, dim3(kSirGrid * 4 / 256), dim3(256), 0, st,
                     (int64_t)kSirGrid * 4, d_wk);
  // kernel timing: for each step between two checks, events before the
  // prefix, after it, after the attempts and after the update
  std::vector<hipEvent_t> ev(phase_ms ? 4 * kSirCheck : 0, nullptr);
  for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  auto elapsed = [&](int i, int j) {
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[i], ev[j]);
    return (double)ms;
  };
  std::vector<SirSim> h_sims((size_t)RB);
  std::vector<int32_t> h_glob((size_t)RB);
  const unsigned gx = sir_blocks(n);
  for (int32_t r0 = 0; r0 < n_sims && e == hipSuccess; r0 += RB) {
    const int32_t R = std::min(RB, n_sims - r0);
    hipLaunchKernelGGL(k_sir_init, dim3(sir_blocks((int64_t)R * n)), dim3(256), 0, st, n, R,
                       state, cand);
    hipLaunchKernelGGL(k_sir_seed, dim3((R + 255) / 256), dim3(256), 0, st, n, R, seed,
                       (int64_t)r0, state, list[0], d_sims, d_nxc);
    int32_t t = 0, pending = 0;  // steps whose events are not read yet
    while (t < t_max) {
      int32_t *cur = list[t & 1], *nxt = list[(t + 1) & 1];
      hipEvent_t *se = phase_ms ? &ev[4 * pending] : nullptr;
      if (se) (void)hipEventRecord(se[0], st);
      hipLaunchKernelGGL(k_sir_prep, dim3(1), dim3(1024), 0, st, R, t, d_sims, d_nxc, d_tabA,
                         d_alive);
      if (se) (void)hipEventRecord(se[1], st);
      hipLaunchKernelGGL(k_sir_attempt, dim3(kSirGrid), dim3(256), 0, st, g.row_ptr, g.col_idx, n,
                         seed, (int64_t)r0, t, tb, R, d_tabA, d_nxc, cur, state, cand, nxt, d_wk);
      if (se) (void)hipEventRecord(se[2], st);
      hipLaunchKernelGGL(k_sir_prep_u, dim3(1), dim3(1024), 0, st, R, d_sims, d_nxc, d_tabU);
      hipLaunchKernelGGL(k_sir_update, dim3(kSirGrid), dim3(256), 0, st, n, seed, (int64_t)r0, t,
                         tm, R, d_tabU, d_nxc, cur, state, nxt);
      if (se) (void)hipEventRecord(se[3], st);
      ++t;
      ++pending;
      if (t % kSirCheck == 0 || t == t_max) {
        // live simulations in the step just run (from its prefix workgroup)
        int32_t alive = 0;
        e = hipMemcpyAsync(&alive, d_alive, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        for (int32_t k = 0; phase_ms && k < pending; ++k) {
          phase_ms[0] += elapsed(4 * k + 1, 4 * k + 2);
          phase_ms[1] += elapsed(4 * k, 4 * k + 1) + elapsed(4 * k + 2, 4 * k + 3);
        }
        pending = 0;
        if (e != hipSuccess || alive == 0) break;
      }
    }
    if (e != hipSuccess) break;
    // fold the last step, then the outcomes of the batch
    hipLaunchKernelGGL(k_sir_prep, dim3(1), dim3(1024), 0, st, R, t, d_sims, d_nxc, d_tabA,
                       d_alive);
    e = hipMemcpyAsync(h_sims.data(), d_sims, sizeof(SirSim) * R, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) break;
    int32_t G = 0;
    for (int32_t r = 0; r < R; ++r) {
      if (work) work[1] += h_sims[r].fsteps;
      index[r0 + r] = h_sims[r].index;
      size[r0 + r] = h_sims[r].size;
      t_end[r0 + r] = h_sims[r].t_end;
      t_peak[r0 + r] = h_sims[r].t_peak;
      if (h_sims[r].size >= global_min) h_glob[G++] = r;
    }
    if (G == 0) continue;
    e = hipMemcpyAsync(d_glob, h_glob.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    // the frontier lists are free now: levels d - 1 and d of the descendant counts
    if (phase_ms) (void)hipEventRecord(ev[0], st);
    for (int d = 1; d <= 4; ++d) {
      int32_t *lc = list[d & 1], *lp = d == 1 ? nullptr : list[(d - 1) & 1];
      hipLaunchKernelGGL(k_sir_zero_rows, dim3(gx, G), dim3(256), 0, st, n, d_glob, lc);
      hipLaunchKernelGGL(k_sir_level, dim3(gx, G), dim3(256), 0, st, n, d_glob, state, cand, lp,
                         lc);
      hipLaunchKernelGGL(k_sir_accum, dim3(gx), dim3(256), 0, st, n, G, d_glob, state, lc,
                         d_sp + (int64_t)(d - 1) * n, d == 1 ? d_ic : nullptr);
    }
    if (phase_ms) {
      e = hipEventRecord(ev[3], st);
      if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
      phase_ms[2] += elapsed(0, 3);
      if (e != hipSuccess) break;
    }
    e = hipStreamSynchronize(st);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(sp_sum, d_sp, sizeof(int64_t) * 4 * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(inf_count, d_ic, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost, st);
  std::vector<int64_t> h_wk(work ? (size_t)kSirGrid * 4 : 0);
  if (e == hipSuccess && work)
    e = hipMemcpyAsync(h_wk.data(), d_wk, sizeof(int64_t) * h_wk.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (int64_t x : h_wk) work[0] += x;
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_status(e, "SIR simulations");
  return EF_OK;
}
