// Triangle pass of the cluster-centric formulation.
//
// Algorithm 1, Phase 2 lowers a cluster's degree by 2 when its two ends are
// adjacent. The pair loop scores every cluster without that adjustment; this
// pass lists every triangle once and records the adjustment:
//   a triangle {x, y, z} with sigma = k_x + k_y + k_z is the node set of three
//   clusters (one per centre); each of its members sees 4 of its event
//   sequences on that node set, so per member the score sum S changes by
//   4 * delta(sigma), delta(sigma) = g(sigma - 6) - g(sigma - 4), and the
//   degree sum D by -8.
// delta is evaluated in registers at each hit (no dependent memory access).
//
// Listing: nodes are ranked by (degree, id); a triangle u < w < x (by rank) is
// found once, at u, as x in up(u) and up(w), where up(.) is the rank-oriented
// out-list. One wavefront per u: up(u) is hashed in LDS (id -> position) and
// the lists up(w), w in up(u), are walked as one concatenated sequence, 64
// consecutive entries per step. Credits:
//   u  - lane registers (floating point), reduced at the end  -> Z[u], ZT[u]
//   w  - LDS add at w's position in up(u)
//   x  - LDS add at x's position in up(u)
// The LDS credit slots hold 64-bit fixed point (2^-40 units), so concurrent
// adds are exact and order-independent: results are bitwise reproducible.
// The slots are written to Y[slot], YT[slot] for the up-arc slots of u.
#include "common.cuh"

namespace efi {

constexpr double kFix = 1099511627776.0;  // 2^40

template <typename T> __device__ __forceinline__ long long to_fix(T v) {
  return __double2ll_rn((double)v * kFix);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// SLOTS: hash slots per wavefront, MAXM: largest |up(u)|, WPB: wavefronts
// per workgroup (each with its own LDS region and its own u).
//
// The lists up(w), w in up(u), are processed as one concatenated sequence:
// non-empty lists are compacted into segments (start in up_col, k_w, w's
// position in up(u)) with an exclusive prefix of their lengths; each step the
// 64 lanes take 64 consecutive entries (coalesced loads, no divergence across
// list lengths) and find their segment by binary search in the prefix.
template <typename T, int SLOTS, int MAXM, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_tri_hash(
    const int32_t *__restrict__ up_ptr, const int32_t *__restrict__ up_col,
    const int32_t *__restrict__ deg, const int32_t *__restrict__ nodes, int64_t count,
    long long *__restrict__ Y, int32_t *__restrict__ YT, void *__restrict__ Z,
    int64_t *__restrict__ ZT) {
  using S = SumT<T>;
  using Acc = typename S::type;
  constexpr int U = 4;  // entries per lane per step (independent loads in flight)
  __shared__ int32_t hkey_s[WPB][SLOTS];
  __shared__ int2 hval_s[WPB][SLOTS];  // (position in up(u), degree)
  __shared__ int32_t seg_w0_s[WPB][MAXM];
  __shared__ int32_t seg_kw_s[WPB][MAXM];
  __shared__ int32_t seg_pos_s[WPB][MAXM];
  __shared__ int32_t seg_p_s[WPB][MAXM + 1];
  __shared__ unsigned long long acc_s[WPB][MAXM];
  __shared__ int32_t accT_s[WPB][MAXM];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t *hkey = hkey_s[wv];
  int2 *hval = hval_s[wv];
  int32_t *seg_w0 = seg_w0_s[wv], *seg_kw = seg_kw_s[wv], *seg_pos = seg_pos_s[wv];
  int32_t *seg_p = seg_p_s[wv];
  unsigned long long *acc = acc_s[wv];
  int32_t *accT = accT_s[wv];
  constexpr int kShift = 32 - __builtin_ctz(SLOTS);
  const unsigned long long lane_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t wave = (int64_t)blockIdx.x * WPB + wv;
  const int64_t nwaves = (int64_t)gridDim.x * WPB;
  for (int64_t it = wave; it < count; it += nwaves) {
    const int32_t u = nodes[it];
    const int32_t u0 = up_ptr[u], m = up_ptr[u + 1] - u0, ku = deg[u];
    for (int i = lane; i < SLOTS; i += 64) hkey[i] = -1;
    for (int i = lane; i < m; i += 64) {
      acc[i] = 0ull;
      accT[i] = 0;
    }
    wave_sync();
    // hash up(u) with each neighbour's degree; compact the non-empty up(w)
    // lists into segments
    int32_t nseg = 0, run = 0;
    for (int c = 0; c < m; c += 64) {
      const int i = c + lane;
      int32_t x = 0, w0 = 0, len = 0, kx = 0;
      if (i < m) {
        x = up_col[u0 + i];
        w0 = up_ptr[x];
        len = up_ptr[x + 1] - w0;
        kx = deg[x];
        uint32_t h = hash32((uint32_t)x) >> kShift;
        while (atomicCAS(&hkey[h], -1, x) != -1) h = (h + 1) & (SLOTS - 1);
        hval[h] = make_int2(i, kx);
      }
      const unsigned long long nz = __ballot(len > 0);
      int32_t incl = len;
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
      }
      if (len > 0) {
        const int slot = nseg + __popcll(nz & lane_mask);
        seg_w0[slot] = w0;
        seg_kw[slot] = kx;
        seg_pos[slot] = i;
        seg_p[slot] = run + incl - len;
      }
      nseg += __popcll(nz);
      run += __shfl(incl, 63, 64);
    }
    if (lane == 0) seg_p[nseg] = run;
    wave_sync();
    const int32_t total = run;
    Acc accu = Acc();
    int64_t cntu = 0;
    for (int32_t base = 0; base < total; base += 64 * U) {
      int32_t xs[U], sg[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int32_t idx = base + q * 64 + lane;
        xs[q] = -2;
        sg[q] = 0;
        if (idx < total) {
          int32_t lo = 0, hi = nseg;  // largest s with seg_p[s] <= idx
          while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (seg_p[mid] <= idx) lo = mid; else hi = mid;
          }
          sg[q] = lo;
          xs[q] = up_col[seg_w0[lo] + (idx - seg_p[lo])];
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int32_t x = xs[q];
        if (x < 0) continue;
        uint32_t h = hash32((uint32_t)x) >> kShift;
        int32_t key;
        while ((key = hkey[h]) != x && key != -1) h = (h + 1) & (SLOTS - 1);
        if (key == x) {
          const int2 pv = hval[h];
          const T dl = tri_delta<T>(ku + seg_kw[sg[q]] + pv.y);
          const unsigned long long f = (unsigned long long)to_fix(dl);
          S::add_term(accu, dl);
          ++cntu;
          atomicAdd(&acc[pv.x], f);
          atomicAdd(&accT[pv.x], 1);
          atomicAdd(&acc[seg_pos[sg[q]]], f);
          atomicAdd(&accT[seg_pos[sg[q]]], 1);
        }
      }
    }
    wave_sync();
    accu = wave_sum(accu);
    cntu = wave_sum_i64(cntu);
    if (lane == 0) {
      S::store(accu, Z, u);
      ZT[u] = cntu;
    }
    for (int i = lane; i < m; i += 64) {
      Y[u0 + i] = (long long)acc[i];
      YT[u0 + i] = accT[i];
    }
    wave_sync();
  }
}

// |up(u)| too long for LDS: membership by binary search in global memory;
// credits go straight to the up-arc slots of u with integer atomics
// (exact, so still order-independent).
template <typename T>
__global__ __launch_bounds__(64) void k_tri_long(const int32_t *__restrict__ up_ptr,
                                                 const int32_t *__restrict__ up_col,
                                                 const int32_t *__restrict__ deg,
                                                 const int32_t *__restrict__ nodes,
                                                 int64_t count, long long *__restrict__ Y,
                                                 int32_t *__restrict__ YT,
                                                 void *__restrict__ Z,
                                                 int64_t *__restrict__ ZT) {
  using S = SumT<T>;
  using Acc = typename S::type;
  const int lane = threadIdx.x;
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t u = nodes[it];
    const int32_t u0 = up_ptr[u], m = up_ptr[u + 1] - u0, ku = deg[u];
    Acc accu = Acc();
    int64_t cntu = 0;
    for (int base = 0; base < m; base += 64) {
      const int i = base + lane;
      int32_t kw = 0, w0 = 0, wl = 0;
      if (i < m) {
        const int32_t w = up_col[u0 + i];
        kw = deg[w];
        w0 = up_ptr[w];
        wl = up_ptr[w + 1] - w0;
      }
      long long accw = 0;
      int32_t cntw = 0;
      for (int32_t j = 0; j < wl; ++j) {
        const int32_t x = up_col[w0 + j];
        int32_t lo = 0, hi = m;
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          if (up_col[u0 + mid] < x) lo = mid + 1; else hi = mid;
        }
        if (lo < m && up_col[u0 + lo] == x) {
          const T dl = tri_delta<T>(ku + kw + deg[x]);
          const long long f = to_fix(dl);
          S::add_term(accu, dl);
          ++cntu;
          accw += f;
          ++cntw;
          atomicAdd((unsigned long long *)&Y[u0 + lo], (unsigned long long)f);
          atomicAdd(&YT[u0 + lo], 1);
        }
      }
      if (cntw) {
        atomicAdd((unsigned long long *)&Y[u0 + i], (unsigned long long)accw);
        atomicAdd(&YT[u0 + i], cntw);
      }
    }
    accu = wave_sum(accu);
    cntu = wave_sum_i64(cntu);
    if (lane == 0) {
      S::store(accu, Z, u);
      ZT[u] = cntu;
    }
  }
}

// zero the outputs of nodes that list no triangle (|up(u)| <= 1) and the
// slots of the long-list nodes (they accumulate with atomics)
template <typename T>
__global__ void k_tri_zero(const int32_t *__restrict__ up_ptr, int32_t n, long long *__restrict__ Y,
                           int32_t *__restrict__ YT, void *__restrict__ Z,
                           int64_t *__restrict__ ZT, int32_t long_min) {
  using S = SumT<T>;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t m = up_ptr[u + 1] - up_ptr[u];
    if (m <= 1) {
      S::store(typename S::type(), Z, u);
      ZT[u] = 0;
    }
    if (m == 1 || m >= long_min) {
      for (int32_t s = up_ptr[u]; s < up_ptr[u + 1]; ++s) {
        Y[s] = 0;
        YT[s] = 0;
      }
    }
  }
}

static unsigned cap_blocks(int64_t b, int64_t cap) {
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

// node lists by |up(u)|: small (2..64), mid (65..512), large (513..2048),
// long (> 2048).
template <typename T>
static hipError_t tri_impl(const Graph &g, const int32_t *const *lists, const int64_t *counts,
                           long long *Y, int32_t *YT, void *Z, int64_t *ZT, hipStream_t st) {
  hipLaunchKernelGGL(k_tri_zero<T>, dim3(cap_blocks((g.n + 255) / 256, 1 << 16)), dim3(256), 0,
                     st, g.up_ptr, g.n, Y, YT, Z, ZT, kTriLongMin);
  if (counts[0] > 0)
    hipLaunchKernelGGL((k_tri_hash<T, 128, 64, 4>), dim3(cap_blocks((counts[0] + 3) / 4, 1 << 20)),
                       dim3(256), 0, st, g.up_ptr, g.up_col, g.deg, lists[0], counts[0], Y, YT,
                       Z, ZT);
  if (counts[1] > 0)
    hipLaunchKernelGGL((k_tri_hash<T, 1024, 512, 2>), dim3(cap_blocks((counts[1] + 1) / 2, 1 << 20)),
                       dim3(128), 0, st, g.up_ptr, g.up_col, g.deg, lists[1], counts[1], Y, YT,
                       Z, ZT);
  if (counts[2] > 0)
    hipLaunchKernelGGL((k_tri_hash<T, 4096, 2048, 1>), dim3(cap_blocks(counts[2], 1 << 20)),
                       dim3(64), 0, st, g.up_ptr, g.up_col, g.deg, lists[2], counts[2], Y, YT,
                       Z, ZT);
  if (counts[3] > 0)
    hipLaunchKernelGGL(k_tri_long<T>, dim3(cap_blocks(counts[3], 1 << 20)), dim3(64), 0, st,
                       g.up_ptr, g.up_col, g.deg, lists[3], counts[3], Y, YT, Z, ZT);
  return hipGetLastError();
}

hipError_t launch_triangles(const Graph &g, ef_prec prec, long long *Y, int32_t *YT, void *Z,
                            int64_t *ZT, hipStream_t st) {
  const int32_t *lists[4] = {g.tri_list[0], g.tri_list[1], g.tri_list[2], g.tri_list[3]};
  if (prec == EF_PREC_FP64) return tri_impl<double>(g, lists, g.n_tri, Y, YT, Z, ZT, st);
  return tri_impl<float>(g, lists, g.n_tri, Y, YT, Z, ZT, st);
}

}  // namespace efi
