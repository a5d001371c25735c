// Triangle pass of the cluster-centric formulation.
//
// Algorithm 1, Phase 2 lowers a cluster's degree by 2 when its two ends are
// adjacent. The pair loop scores every cluster without that adjustment; this
// pass lists every triangle once and records the adjustment:
//   a triangle {x, y, z} with sigma = k_x + k_y + k_z is the node set of three
//   clusters (one per centre); each of its members sees 4 of its event
//   sequences on that node set, so per member the score sum S changes by
//   4 * (g(sigma - 6) - g(sigma - 4)) and the degree sum D by -8.
//
// Listing: nodes are ranked by (degree, id); a triangle u < w < x (by rank) is
// found once, at u, as x in up(u) and up(w), where up(.) is the rank-oriented
// out-list. One wavefront per u: up(u) is hashed in LDS; the wavefront walks
// w over up(u) and its lanes walk x over up(w). Credits go to
//   u  - lane registers, reduced at the end               -> Z[u], ZT[u]
//   w  - wavefront sum per w, into LDS by position in up(u)
//   x  - into LDS by position in up(u); lanes of one step hold distinct x
// and the LDS sums are written to Y[slot], YT[slot] for the up-arc slots of
// u. Every accumulation happens in a fixed order, so results are reproducible.
#include "common.cuh"

namespace efi {

template <typename T, int SLOTS, int MAXM>
__global__ __launch_bounds__(64) void k_tri_hash(const int32_t *__restrict__ up_ptr,
                                                 const int32_t *__restrict__ up_col,
                                                 const int32_t *__restrict__ deg,
                                                 const int32_t *__restrict__ nodes,
                                                 int64_t count, void *__restrict__ Y,
                                                 int32_t *__restrict__ YT,
                                                 void *__restrict__ Z,
                                                 int64_t *__restrict__ ZT) {
  using S = SumT<T>;
  using Acc = typename S::type;
  __shared__ int32_t hkey[SLOTS];
  __shared__ int32_t hpos[SLOTS];
  __shared__ int32_t hdeg[SLOTS];
  __shared__ Acc acc[MAXM];
  __shared__ int32_t accT[MAXM];
  const int lane = threadIdx.x;
  constexpr int kShift = 32 - __builtin_ctz(SLOTS);
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t u = nodes[it];
    const int32_t u0 = up_ptr[u], m = up_ptr[u + 1] - u0, ku = deg[u];
    for (int i = lane; i < SLOTS; i += 64) hkey[i] = -1;
    for (int i = lane; i < m; i += 64) {
      acc[i] = Acc();
      accT[i] = 0;
    }
    __syncthreads();
    for (int i = lane; i < m; i += 64) {
      const int32_t x = up_col[u0 + i];
      uint32_t h = hash32((uint32_t)x) >> kShift;
      while (true) {
        int32_t prev = atomicCAS(&hkey[h], -1, x);
        if (prev == -1) {
          hpos[h] = i;
          hdeg[h] = deg[x];
          break;
        }
        h = (h + 1) & (SLOTS - 1);
      }
    }
    __syncthreads();
    Acc accu = Acc();
    int64_t cntu = 0;
    for (int i = 0; i < m; ++i) {
      const int32_t w = up_col[u0 + i];
      const int32_t kw = deg[w];
      const int32_t w0 = up_ptr[w], wm = up_ptr[w + 1] - w0;
      Acc accw = Acc();
      int32_t cntw = 0;
      for (int j = lane; j < wm; j += 64) {
        const int32_t x = up_col[w0 + j];
        uint32_t h = hash32((uint32_t)x) >> kShift;
        int32_t pos = -1, kx = 0;
        while (true) {
          const int32_t key = hkey[h];
          if (key == x) {
            pos = hpos[h];
            kx = hdeg[h];
            break;
          }
          if (key == -1) break;
          h = (h + 1) & (SLOTS - 1);
        }
        if (pos >= 0) {
          const T dl = tri_delta<T>(ku + kw + kx);
          S::add_term(accu, dl);
          S::add_term(accw, dl);
          ++cntu;
          ++cntw;
          S::add_term(acc[pos], dl);
          accT[pos] += 1;
        }
      }
      __syncthreads();
      accw = wave_sum(accw);
      cntw = (int32_t)wave_sum_i64(cntw);
      if (lane == 0 && cntw) {
        S::add_term(acc[i], S::value(accw));
        accT[i] += cntw;
      }
      __syncthreads();
    }
    accu = wave_sum(accu);
    cntu = wave_sum_i64(cntu);
    if (lane == 0) {
      S::store(accu, Z, u);
      ZT[u] = cntu;
    }
    for (int i = lane; i < m; i += 64) {
      S::store(acc[i], Y, u0 + i);
      YT[u0 + i] = accT[i];
    }
    __syncthreads();
  }
}

// up(u) too long for LDS: binary search in global memory, credits to the
// up-arc slots of u with atomics (rare: only when |up(u)| > 4096).
template <typename T>
__global__ __launch_bounds__(64) void k_tri_long(const int32_t *__restrict__ up_ptr,
                                                 const int32_t *__restrict__ up_col,
                                                 const int32_t *__restrict__ deg,
                                                 const int32_t *__restrict__ nodes,
                                                 int64_t count, T *__restrict__ Yacc,
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
    for (int i = 0; i < m; ++i) {
      const int32_t w = up_col[u0 + i];
      const int32_t kw = deg[w];
      const int32_t w0 = up_ptr[w], wm = up_ptr[w + 1] - w0;
      T accw = T(0);
      int32_t cntw = 0;
      for (int j = lane; j < wm; j += 64) {
        const int32_t x = up_col[w0 + j];
        int32_t lo = 0, hi = m;
        while (lo < hi) {
          int32_t mid = (lo + hi) >> 1;
          if (up_col[u0 + mid] < x) lo = mid + 1; else hi = mid;
        }
        if (lo < m && up_col[u0 + lo] == x) {
          const T dl = tri_delta<T>(ku + kw + deg[x]);
          S::add_term(accu, dl);
          accw += dl;
          ++cntu;
          ++cntw;
          atomicAdd(&Yacc[u0 + lo], dl);
          atomicAdd(&YT[u0 + lo], 1);
        }
      }
      accw = wave_sum(accw);
      cntw = (int32_t)wave_sum_i64(cntw);
      if (lane == 0 && cntw) {
        atomicAdd(&Yacc[u0 + i], accw);
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

// The long path accumulates plain T per slot; convert into the slot layout.
template <typename T>
__global__ void k_tri_long_store(const int32_t *__restrict__ up_ptr,
                                 const int32_t *__restrict__ nodes, int64_t count,
                                 const T *__restrict__ Yacc, void *__restrict__ Y) {
  using S = SumT<T>;
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t u = nodes[it];
    for (int32_t s = up_ptr[u] + threadIdx.x; s < up_ptr[u + 1]; s += blockDim.x) {
      typename S::type a = typename S::type();
      S::add_term(a, Yacc[s]);
      S::store(a, Y, s);
    }
  }
}

// zero the outputs of nodes that list no triangle (|up(u)| <= 1)
template <typename T>
__global__ void k_tri_zero(const int32_t *__restrict__ up_ptr, int32_t n, void *__restrict__ Y,
                           int32_t *__restrict__ YT, void *__restrict__ Z,
                           int64_t *__restrict__ ZT) {
  using S = SumT<T>;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t m = up_ptr[u + 1] - up_ptr[u];
    if (m <= 1) {
      S::store(typename S::type(), Z, u);
      ZT[u] = 0;
      if (m == 1) {
        S::store(typename S::type(), Y, up_ptr[u]);
        YT[up_ptr[u]] = 0;
      }
    }
  }
}

// clear the up-arc slots of the long-path nodes (only their own slots)
template <typename T>
__global__ void k_tri_long_clear(const int32_t *__restrict__ up_ptr,
                                 const int32_t *__restrict__ nodes, int64_t count,
                                 T *__restrict__ Yacc, int32_t *__restrict__ YT) {
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t u = nodes[it];
    for (int32_t s = up_ptr[u] + threadIdx.x; s < up_ptr[u + 1]; s += blockDim.x) {
      Yacc[s] = T(0);
      YT[s] = 0;
    }
  }
}

static unsigned cap_blocks(int64_t b, int64_t cap) {
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

// node lists: hash_small (|up| in [2, 512]), hash_large (|up| in (512, 4096]),
// long (|up| > 4096). Yacc_tmp: up-arc-sized T scratch for the long path.
template <typename T>
static hipError_t tri_impl(const Graph &g, const int32_t *small, int64_t n_small,
                           const int32_t *large, int64_t n_large, const int32_t *lng,
                           int64_t n_long, void *Y, int32_t *YT, void *Z, int64_t *ZT,
                           T *Yacc_tmp, hipStream_t st) {
  hipLaunchKernelGGL(k_tri_zero<T>, dim3(cap_blocks((g.n + 255) / 256, 1 << 16)), dim3(256), 0,
                     st, g.up_ptr, g.n, Y, YT, Z, ZT);
  if (n_small > 0)
    hipLaunchKernelGGL((k_tri_hash<T, kTriHashSlots, kTriHashMax>),
                       dim3(cap_blocks(n_small, 1 << 20)), dim3(64), 0, st, g.up_ptr, g.up_col,
                       g.deg, small, n_small, Y, YT, Z, ZT);
  if (n_large > 0)
    hipLaunchKernelGGL((k_tri_hash<T, 8192, 4096>), dim3(cap_blocks(n_large, 1 << 20)), dim3(64),
                       0, st, g.up_ptr, g.up_col, g.deg, large, n_large, Y, YT, Z, ZT);
  if (n_long > 0) {
    hipLaunchKernelGGL(k_tri_long_clear<T>, dim3(cap_blocks(n_long, 1 << 16)), dim3(256), 0, st,
                       g.up_ptr, lng, n_long, Yacc_tmp, YT);
    hipLaunchKernelGGL(k_tri_long<T>, dim3(cap_blocks(n_long, 1 << 20)), dim3(64), 0, st,
                       g.up_ptr, g.up_col, g.deg, lng, n_long, Yacc_tmp, YT, Z, ZT);
    hipLaunchKernelGGL(k_tri_long_store<T>, dim3(cap_blocks(n_long, 1 << 16)), dim3(256), 0, st,
                       g.up_ptr, lng, n_long, Yacc_tmp, Y);
  }
  return hipGetLastError();
}

hipError_t launch_triangles_ex(const Graph &g, ef_prec prec, const int32_t *small,
                               int64_t n_small, const int32_t *large, int64_t n_large,
                               const int32_t *lng, int64_t n_long, void *Y, int32_t *YT,
                               void *Z, int64_t *ZT, void *Yacc_tmp, hipStream_t st) {
  if (prec == EF_PREC_FP64)
    return tri_impl<double>(g, small, n_small, large, n_large, lng, n_long, Y, YT, Z, ZT,
                            (double *)Yacc_tmp, st);
  return tri_impl<float>(g, small, n_small, large, n_large, lng, n_long, Y, YT, Z, ZT,
                         (float *)Yacc_tmp, st);
}

}  // namespace efi
