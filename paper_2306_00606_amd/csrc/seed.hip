// Per-node sums and Eq. 1; the per-seed formulation's 2-hop stream; the FP32
// recomputation pass for cancellation-prone seeds; output scatter.
//
// With R[v->a] = sum over the clusters centred at v that contain a of g(d)
// (before the triangle adjustment), a seed s collects
//   S(s) = sum_{a in N(s)} (R[s->a] + R[a->s]) + 4 * sum_{triangles t at s} delta(t)
// because every cluster credited to s is either centred at s (the row sums
// of its own arcs; stars, reached twice) or centred at a neighbour a with s
// as an end (the row sum of the reverse arc; paths, reached once).
// N(s) and D(s) follow the same split with exact integer sums:
//   per arc v->a:  N = k_v - 1,   D = (k_v - 1)(k_v + k_a - 4) + (A_v - k_a)
// (A_v = sum of v's neighbour degrees), minus 8 per triangle at s for D.
// Then EF(s) = ln D - S / D (Eq. 1 with p_c = d_c / D).
#include "common.cuh"

namespace efi {

constexpr double kLn2 = 0.69314718055994530942;

// Eq. 1 from the sums; appends cancellation-prone FP32 results to `flagged`.
template <typename T>
__device__ __forceinline__ double finish_ef(int64_t Nn, int64_t Dd, double S, int32_t pos,
                                           int32_t *flagged, int32_t *flag_count,
                                           int32_t *fp64_count);

template <>
__device__ __forceinline__ double finish_ef<double>(int64_t Nn, int64_t Dd, double S, int32_t,
                                                   int32_t *, int32_t *, int32_t *) {
  if (Dd <= 0 || Nn <= 1) return 0.0;
  const double ef = log((double)Dd) - S / (double)Dd;
  return ef > 0.0 ? ef : 0.0;
}

// FP32 path: S in log2 units (double-float, passed as its double value).
template <>
__device__ __forceinline__ double finish_ef<float>(int64_t Nn, int64_t Dd, double S2, int32_t pos,
                                                  int32_t *flagged, int32_t *flag_count,
                                                  int32_t *fp64_count) {
  if (Dd <= 0 || Nn <= 1) return 0.0;
  double ef;
  float mu, e32;
  if (Nn > (1LL << 24)) {
    // more than 2^24 clusters: final combination in double precision
    const double mu_d = S2 / (double)Dd;
    const double e2 = log2((double)Dd) - mu_d;
    ef = kLn2 * e2;
    mu = (float)mu_d;
    e32 = (float)e2;
    atomicAdd(fp64_count, 1);
  } else {
    const float Df = (float)Dd;
    mu = (float)S2 / Df;
    e32 = log2f(Df) - mu;
    ef = kLn2 * (double)e32;
  }
  if (!(e32 > 0.0f) || mu > kKappaMax * e32) {
    flagged[atomicAdd(flag_count, 1)] = pos;
  }
  return ef > 0.0 ? ef : 0.0;
}

// ---------------------------------------------------------------------------
// cluster-centric: one wavefront per node
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_finalize_cluster(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ deg,
    const int2 *__restrict__ adj2, const int32_t *__restrict__ rev,
    const int32_t *__restrict__ tslot, const int64_t *__restrict__ asum,
    const void *__restrict__ R, const long long *__restrict__ Y, const int32_t *__restrict__ YT,
    const void *__restrict__ Z, const int64_t *__restrict__ ZT, int32_t n,
    double *__restrict__ ef, int64_t *__restrict__ Dout, int64_t *__restrict__ Nout,
    int32_t *__restrict__ flagged, int32_t *__restrict__ flag_count,
    int32_t *__restrict__ fp64_count) {
  using S = SumT<T>;
  using Acc = typename S::type;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int32_t k = deg[v], base = row_ptr[v];
    const int64_t As = asum[v];
    Acc sacc = Acc();
    double tfix = 0.0;  // triangle credits, 2^-40 fixed-point units
    int64_t Nn = 0, Dd = 0, Tc = 0;
    for (int32_t e = base + lane; e < base + k; e += 64) {
      const int2 ad = adj2[e];
      const int32_t a = ad.x, ka = ad.y;
      // a centre of degree 1 has no pairs: its row sums were never written
      if (k >= 2) S::add_stored(sacc, R, e);
      if (ka >= 2) S::add_stored(sacc, R, rev[e]);
      Nn += (int64_t)(k - 1) + (ka - 1);
      Dd += (int64_t)(k - 1) * (k + ka - 4) + (As - ka) + (int64_t)(ka - 1) * (ka + k - 4) +
            (asum[a] - k);
      if (rank_less_d(a, ka, (int32_t)v, k)) {
        const int32_t sl = tslot[e];
        tfix += (double)Y[sl];
        Tc += YT[sl];
      }
    }
    sacc = wave_sum(sacc);
    tfix = wave_sum_f64(tfix);
    Nn = wave_sum_i64(Nn);
    Dd = wave_sum_i64(Dd);
    Tc = wave_sum_i64(Tc);
    if (lane == 0) {
      Acc z = Acc();
      S::add_stored(z, Z, v);
      Tc += ZT[v];
      const double tri = tfix * (1.0 / 1099511627776.0) + S::value(z);
      const double Stot = S::value(sacc) + 4.0 * tri;
      Dd -= 8 * Tc;
      ef[v] = finish_ef<T>(Nn, Dd, Stot, (int32_t)v, flagged, flag_count, fp64_count);
      Dout[v] = Dd;
      Nout[v] = Nn;
    }
  }
}

static unsigned cap_blocks(int64_t b, int64_t cap) {
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

hipError_t launch_finalize_cluster(const Graph &g, ef_prec prec, const void *R,
                                   const long long *Y, const int32_t *YT, const void *Z, const int64_t *ZT,
                                   double *ef, int64_t *D, int64_t *N, int32_t *flagged,
                                   int32_t *flag_count, int32_t *fp64_count, hipStream_t st) {
  const unsigned blocks = cap_blocks(((int64_t)g.n * 64 + 255) / 256, 1 << 20);
  if (prec == EF_PREC_FP64)
    hipLaunchKernelGGL(k_finalize_cluster<double>, dim3(blocks), dim3(256), 0, st, g.row_ptr,
                       g.deg, g.adj2, g.rev, g.tslot, g.asum, R, Y, YT, Z, ZT, g.n, ef, D, N,
                       flagged, flag_count, fp64_count);
  else
    hipLaunchKernelGGL(k_finalize_cluster<float>, dim3(blocks), dim3(256), 0, st, g.row_ptr,
                       g.deg, g.adj2, g.rev, g.tslot, g.asum, R, Y, YT, Z, ZT, g.n, ef, D, N,
                       flagged, flag_count, fp64_count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// block helpers
// ---------------------------------------------------------------------------
template <typename A>
__device__ A block_sum_acc(A x, A *sh) {
  // 256 threads: wavefront sums, then lane 0 of wavefront 0 adds 4 values in order
  x = wave_sum(x);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[w] = x;
  __syncthreads();
  A r = sh[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) acc_merge(r, sh[i]);
  __syncthreads();
  return r;
}
__device__ int64_t block_sum_i64(int64_t x, int64_t *sh) {
  x = wave_sum_i64(x);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[w] = x;
  __syncthreads();
  int64_t r = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// per-seed formulation: star sums from R over the seed's own arcs, paths and
// the star triangle adjustment from the 2-hop stream, membership in N(s) from
// an LDS hash (k <= 2048) or a device bitmap.
// ---------------------------------------------------------------------------
__global__ void k_bitmap_set(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                             const int32_t *__restrict__ big_seeds, int32_t n_big,
                             uint32_t *__restrict__ bm, int64_t words, int set) {
  for (int32_t bi = blockIdx.x; bi < n_big; bi += gridDim.x) {
    const int32_t s = big_seeds[bi];
    uint32_t *b = bm + (int64_t)bi * words;
    for (int32_t e = row_ptr[s] + threadIdx.x; e < row_ptr[s + 1]; e += blockDim.x) {
      const int32_t x = col[e];
      if (set) atomicOr(&b[x >> 5], 1u << (x & 31));
      else b[x >> 5] = 0u;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_seed_stream(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ deg,
    const int2 *__restrict__ adj2, const int64_t *__restrict__ asum,
    const int32_t *__restrict__ seeds, int32_t n_seeds, const void *__restrict__ R,
    const uint32_t *__restrict__ bm, const int32_t *__restrict__ big_slot, int64_t words,
    double *__restrict__ ef, int64_t *__restrict__ Dout, int64_t *__restrict__ Nout,
    int32_t *__restrict__ flagged, int32_t *__restrict__ flag_count,
    int32_t *__restrict__ fp64_count) {
  using S = SumT<T>;
  using Acc = typename S::type;
  __shared__ int32_t hkey[kSeedHashSlots];
  __shared__ int32_t pref[257];
  __shared__ int32_t arow[256], aid[256], ak[256];
  __shared__ Acc shA[4];
  __shared__ int64_t shI[4];
  constexpr int kShift = 32 - __builtin_ctz(kSeedHashSlots);
  const int tid = threadIdx.x;
  for (int32_t it = blockIdx.x; it < n_seeds; it += gridDim.x) {
    const int32_t s = seeds[it];
    const int32_t k = deg[s], base = row_ptr[s];
    const int32_t bslot = big_slot ? big_slot[it] : -1;
    const uint32_t *mybm = bslot >= 0 ? bm + (int64_t)bslot * words : nullptr;
    if (!mybm) {
      for (int i = tid; i < kSeedHashSlots; i += 256) hkey[i] = -1;
      __syncthreads();
      for (int e = base + tid; e < base + k; e += 256) {
        const int32_t x = adj2[e].x;
        uint32_t h = hash32((uint32_t)x) >> kShift;
        while (atomicCAS(&hkey[h], -1, x) != -1) h = (h + 1) & (kSeedHashSlots - 1);
      }
      __syncthreads();
    }
    Acc sacc = Acc();
    int64_t Dd = 0, Nn = 0;
    if (k >= 2)
      for (int e = base + tid; e < base + k; e += 256) S::add_stored(sacc, R, e);
    for (int32_t c0 = 0; c0 < k; c0 += 256) {
      const int32_t cnt = min(256, k - c0);
      int32_t len = 0;
      if (tid < cnt) {
        const int2 ad = adj2[base + c0 + tid];
        aid[tid] = ad.x;
        ak[tid] = ad.y;
        arow[tid] = row_ptr[ad.x];
        len = ad.y;
      }
      // block exclusive scan of len into pref
      {
        const int lane = tid & 63, w = tid >> 6;
        int32_t incl = len;
        for (int off = 1; off < 64; off <<= 1) {
          int32_t y = __shfl_up(incl, off, 64);
          if (lane >= off) incl += y;
        }
        __shared__ int32_t wsum[4];
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int32_t woff = 0;
        for (int i = 0; i < w; ++i) woff += wsum[i];
        pref[tid] = woff + incl - len;
        if (tid == 255) pref[256] = woff + incl;
        __syncthreads();
      }
      const int32_t total = pref[256];
      for (int32_t idx = tid; idx < total; idx += 256) {
        int32_t lo = 0, hi = cnt;  // largest j with pref[j] <= idx
        while (hi - lo > 1) {
          int32_t mid = (lo + hi) >> 1;
          if (pref[mid] <= idx) lo = mid; else hi = mid;
        }
        const int32_t ka = ak[lo];
        const int2 bd = adj2[arow[lo] + (idx - pref[lo])];
        const int32_t b = bd.x, kb = bd.y;
        if (b == s) continue;
        bool m;
        if (mybm) {
          m = (mybm[b >> 5] >> (b & 31)) & 1u;
        } else {
          uint32_t h = hash32((uint32_t)b) >> kShift;
          m = false;
          while (true) {
            const int32_t key = hkey[h];
            if (key == b) { m = true; break; }
            if (key == -1) break;
            h = (h + 1) & (kSeedHashSlots - 1);
          }
        }
        const int32_t sigma = k + ka + kb;
        const int32_t d = sigma - 4 - (m ? 2 : 0);
        S::add_term(sacc, score_t<T>(d));
        Dd += d;
        Nn += 1;
        if (m) {
          // star (a, b) with a ~ b: the pair loop scored it with degree sigma - 4
          S::add_term(sacc, tri_delta<T>(sigma));
          Dd -= 2;
        }
      }
      __syncthreads();
    }
    sacc = block_sum_acc(sacc, shA);
    Dd = block_sum_i64(Dd, shI);
    Nn = block_sum_i64(Nn, shI);
    if (tid == 0) {
      const int64_t kk = k;
      const int64_t As = asum[s];
      Nn += kk * (kk - 1);
      Dd += kk * (kk - 1) * (kk - 4) + 2 * (kk - 1) * As;
      ef[it] = finish_ef<T>(Nn, Dd, S::value(sacc), it, flagged, flag_count, fp64_count);
      Dout[it] = Dd;
      Nout[it] = Nn;
    }
    __syncthreads();
  }
}

hipError_t launch_per_seed(const Graph &g, ef_prec prec, const int32_t *seeds, int32_t n_seeds,
                           const void *R, uint32_t *bitmaps, const int32_t *big_seeds,
                           const int32_t *big_slot, int32_t n_big_seeds, double *ef, int64_t *D,
                           int64_t *N, int32_t *flagged, int32_t *flag_count,
                           int32_t *fp64_count, hipStream_t st, hipEvent_t ev_stream_done) {
  const int64_t words = ((int64_t)g.n + 31) / 32;
  if (n_big_seeds > 0)
    hipLaunchKernelGGL(k_bitmap_set, dim3(cap_blocks(n_big_seeds, 65536)), dim3(256), 0, st,
                       g.row_ptr, g.col_idx, big_seeds, n_big_seeds, bitmaps, words, 1);
  const unsigned blocks = cap_blocks(n_seeds, 1 << 20);
  if (prec == EF_PREC_FP64)
    hipLaunchKernelGGL(k_seed_stream<double>, dim3(blocks), dim3(256), 0, st, g.row_ptr, g.deg,
                       g.adj2, g.asum, seeds, n_seeds, R, bitmaps,
                       n_big_seeds > 0 ? big_slot : nullptr, words, ef, D, N, flagged,
                       flag_count, fp64_count);
  else
    hipLaunchKernelGGL(k_seed_stream<float>, dim3(blocks), dim3(256), 0, st, g.row_ptr, g.deg,
                       g.adj2, g.asum, seeds, n_seeds, R, bitmaps,
                       n_big_seeds > 0 ? big_slot : nullptr, words, ef, D, N, flagged,
                       flag_count, fp64_count);
  if (ev_stream_done) (void)hipEventRecord(ev_stream_done, st);
  if (n_big_seeds > 0)
    hipLaunchKernelGGL(k_bitmap_set, dim3(cap_blocks(n_big_seeds, 65536)), dim3(256), 0, st,
                       g.row_ptr, g.col_idx, big_seeds, n_big_seeds, bitmaps, words, 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 pass 2: EF = (1/D) sum_c d_c log1p((D - d_c) / d_c), every term >= 0,
// for seeds whose ln D - S/D form loses accuracy to cancellation. D is the
// exact value from pass 1. Stars need the adjacency of their two ends: for
// k <= 512 a bit matrix over N(s) x N(s) in LDS, filled from the path stream;
// otherwise a binary search in the end's row.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float term_nonneg(int32_t d, int64_t D) {
  if (d <= 0) return 0.0f;
  const float df = (float)d;
  return df * log1pf((float)(D - d) / df);
}

__device__ __forceinline__ int32_t find_sorted(const int32_t *a, int32_t len, int32_t x) {
  int32_t lo = 0, hi = len;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return (lo < len && a[lo] == x) ? lo : -1;
}

constexpr int kP2Max = 512;

__global__ __launch_bounds__(256) void k_pass2(const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col,
                                               const int32_t *__restrict__ deg,
                                               const int2 *__restrict__ adj2,
                                               const int32_t *__restrict__ seeds,
                                               const int32_t *__restrict__ flagged,
                                               const int32_t *__restrict__ flag_count,
                                               double *__restrict__ ef,
                                               const int64_t *__restrict__ Dv) {
  __shared__ int32_t nid[kP2Max], nk[kP2Max];
  __shared__ uint32_t bits[kP2Max * (kP2Max / 32)];
  __shared__ DFv shA[4];
  const int tid = threadIdx.x;
  const int32_t count = *flag_count;
  for (int32_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t pos = flagged[it];
    const int32_t s = seeds ? seeds[pos] : pos;
    const int32_t k = deg[s], base = row_ptr[s];
    const int64_t D = Dv[pos];
    const bool lds = k <= kP2Max;
    constexpr int W = kP2Max / 32;
    if (lds) {
      for (int i = tid; i < k; i += 256) {
        const int2 ad = adj2[base + i];
        nid[i] = ad.x;
        nk[i] = ad.y;
      }
      for (int i = tid; i < k * W; i += 256) bits[i] = 0u;
    }
    __syncthreads();
    DFv acc = DFv();
    // paths s -> a -> b (one event order each)
    for (int32_t i = 0; i < k; ++i) {
      const int2 ad = adj2[base + i];
      const int32_t a = ad.x, ka = ad.y;
      for (int32_t f = row_ptr[a] + tid; f < row_ptr[a + 1]; f += 256) {
        const int2 bd = adj2[f];
        const int32_t b = bd.x;
        if (b == s) continue;
        const int32_t j = lds ? find_sorted(nid, k, b) : find_sorted(col + base, k, b);
        if (j >= 0 && lds) atomicOr(&bits[i * W + (j >> 5)], 1u << (j & 31));
        acc.add(term_nonneg(k + ka + bd.y - 4 - (j >= 0 ? 2 : 0), D));
      }
    }
    __syncthreads();
    // stars a - s - b (two event orders each)
    for (int32_t i = 0; i < k; ++i) {
      const int32_t a = lds ? nid[i] : adj2[base + i].x;
      const int32_t ka = lds ? nk[i] : adj2[base + i].y;
      for (int32_t j = i + 1 + tid; j < k; j += 256) {
        const int32_t kb = lds ? nk[j] : adj2[base + j].y;
        bool m;
        if (lds) m = (bits[i * W + (j >> 5)] >> (j & 31)) & 1u;
        else m = find_sorted(col + row_ptr[a], deg[a], col[base + j]) >= 0;
        const float t = term_nonneg(k + ka + kb - 4 - (m ? 2 : 0), D);
        acc.add(t);
        acc.add(t);
      }
    }
    acc = block_sum_acc(acc, shA);
    if (tid == 0) {
      const double e = acc.value() / (double)D;
      ef[pos] = e > 0.0 ? e : 0.0;
    }
    __syncthreads();
  }
}

hipError_t launch_pass2(const Graph &g, const int32_t *seeds, const int32_t *flagged,
                        const int32_t *flag_count, int32_t max_flagged, double *ef,
                        const int64_t *D, hipStream_t st) {
  if (max_flagged <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pass2, dim3(cap_blocks(max_flagged, 8192)), dim3(256), 0, st, g.row_ptr,
                     g.col_idx, g.deg, g.adj2, seeds, flagged, flag_count, ef, D);
  return hipGetLastError();
}

__global__ void k_gather_out(const int32_t *__restrict__ inv, int32_t count,
                             const double *__restrict__ ef_u, const int64_t *__restrict__ D_u,
                             const int64_t *__restrict__ N_u, double *__restrict__ ef,
                             int64_t *__restrict__ D, int64_t *__restrict__ N) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = inv[i];
    ef[i] = ef_u[u];
    if (D) D[i] = D_u[u];
    if (N) N[i] = N_u[u];
  }
}

hipError_t launch_gather_outputs(const int32_t *inv, int32_t count, const double *ef_u,
                                 const int64_t *D_u, const int64_t *N_u, double *ef, int64_t *D,
                                 int64_t *N, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_out, dim3(cap_blocks((count + 255) / 256, 65536)), dim3(256), 0,
                     st, inv, count, ef_u, D_u, N_u, ef, D, N);
  return hipGetLastError();
}

}  // namespace efi
