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
#include "device_common.h"

namespace efi {

constexpr double kLn2 = 0.69314718055994530942;

// Eq. 1 from the sums. fl[pos] receives the position's flags: bit 0 the
// FP32 result is cancellation-prone (recomputed by pass 2), bit 1 it was
// finalised in FP64 (more than 2^24 clusters). Flags are bytes, compacted
// afterwards by k_flag_compact: no contended atomics here.
template <typename T>
__device__ __forceinline__ double finish_ef(int64_t Nn, int64_t Dd, double S, int32_t pos,
                                           uint8_t *fl);

template <>
__device__ __forceinline__ double finish_ef<double>(int64_t Nn, int64_t Dd, double S, int32_t pos,
                                                   uint8_t *fl) {
  fl[pos] = 0;
  if (Dd <= 0 || Nn <= 1) return 0.0;
  const double ef = log((double)Dd) - S / (double)Dd;
  return ef > 0.0 ? ef : 0.0;
}

// FP32 path: S in log2 units (double-float, passed as its double value).
template <>
__device__ __forceinline__ double finish_ef<float>(int64_t Nn, int64_t Dd, double S2, int32_t pos,
                                                  uint8_t *fl) {
  if (Dd <= 0 || Nn <= 1) {
    fl[pos] = 0;
    return 0.0;
  }
  double ef;
  float mu, e32;
  uint8_t f = 0;
  if (Nn > (1LL << 24)) {
    // more than 2^24 clusters: final combination in double precision
    const double mu_d = S2 / (double)Dd;
    const double e2 = log2((double)Dd) - mu_d;
    ef = kLn2 * e2;
    mu = (float)mu_d;
    e32 = (float)e2;
    f |= 2;
  } else {
    const float Df = (float)Dd;
    mu = (float)S2 / Df;
    e32 = log2f(Df) - mu;
    ef = kLn2 * (double)e32;
  }
  if (!(e32 > 0.0f) || mu > kKappaMax * e32) f |= 1;
  fl[pos] = f;
  return ef > 0.0 ? ef : 0.0;
}

// Compact the flag bytes of positions 0..n-1: positions with bit 0 go to
// `flagged` (counts[0] of them), bit 1 is counted in counts[1]. Each
// workgroup owns a contiguous range and takes one atomic per counter.
__global__ __launch_bounds__(1024) void k_flag_compact(const uint8_t *__restrict__ fl, int64_t n,
                                                       int32_t *__restrict__ flagged,
                                                       int32_t *__restrict__ counts) {
  __shared__ int32_t wa[16], wb[16];
  __shared__ int32_t base_s;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  int32_t c = 0, f = 0;
  for (int64_t i = lo + tid; i < hi; i += 1024) {
    const uint8_t x = fl[i];
    c += x & 1;
    f += (x >> 1) & 1;
  }
  for (int off = 32; off > 0; off >>= 1) {
    c += __shfl_xor(c, off, 64);
    f += __shfl_xor(f, off, 64);
  }
  if (lane == 0) {
    wa[wv] = c;
    wb[wv] = f;
  }
  __syncthreads();
  if (tid == 0) {
    int32_t ct = 0, ft = 0;
    for (int w = 0; w < 16; ++w) {
      ct += wa[w];
      ft += wb[w];
    }
    base_s = ct ? atomicAdd(&counts[0], ct) : 0;
    if (ft) atomicAdd(&counts[1], ft);
  }
  __syncthreads();
  int32_t run = base_s;
  for (int64_t i0 = lo; i0 < hi; i0 += 1024) {
    const int64_t i = i0 + tid;
    const bool p = i < hi && (fl[i] & 1);
    const unsigned long long m = __ballot(p);
    if (lane == 0) wa[wv] = __popcll(m);
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wv) pre += wa[w];
      tot += wa[w];
    }
    if (p) flagged[run + pre + __popcll(m & below)] = (int32_t)i;
    run += tot;
    __syncthreads();
  }
}

hipError_t launch_flag_compact(const uint8_t *fl, int64_t n, int32_t *flagged, int32_t *counts,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 4095) / 4096;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(k_flag_compact, dim3((unsigned)blocks), dim3(1024), 0, st, fl, n, flagged,
                     counts);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cluster-centric finalize: G lanes per node. nodes == nullptr: nodes
// 0..count-1 of degree <= kmax; otherwise the listed nodes.
// ---------------------------------------------------------------------------
template <int G> __device__ __forceinline__ int64_t group_sum(int64_t x) {
  for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, G);
  return x;
}
template <int G> __device__ __forceinline__ double group_sum(double x) {
  for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, G);
  return x;
}
template <int G> __device__ __forceinline__ DFv group_sum(DFv x) {
  for (int off = G / 2; off > 0; off >>= 1) {
    DFv o;
    o.hi = __shfl_xor(x.hi, off, G);
    o.lo = __shfl_xor(x.lo, off, G);
    x.add(o);
  }
  return x;
}

// arcs first, first + stride, ... of node v: its own row sums R[e], the
// reverse arcs' sums R[rrev e] (a big centre keeps its row's sums in sorted
// order, so its own sum over the row is the same set), and the triangle
// credits to v kept with each of its edges (record trec[e]; -1: no walk wrote
// one, nothing to add)
template <typename T>
__device__ __forceinline__ void fin_arcs(const int2 *__restrict__ adj2,
                                         const int32_t *__restrict__ rrev,
                                         const int32_t *__restrict__ trec, const void *R,
                                         const TriSlot *__restrict__ Y, int32_t k, int32_t base,
                                         int32_t first, int32_t stride,
                                         typename SumT<T>::type &sacc, double &tfix,
                                         int64_t &Tc) {
  using S = SumT<T>;
  for (int32_t e = base + first; e < base + k; e += stride) {
    // a centre of degree 1 has no pairs: its row sums were never written
    if (k >= 2) S::add_arc(sacc, R, e);
    if (adj2[e].y >= 2) S::add_arc(sacc, R, rrev[e]);
    const int32_t r = trec[e];
    if (r >= 0) {
      const TriSlot t = Y[r];
      tfix += (double)t.y;  // 2^-36 fixed-point units
      Tc += t.t;
    }
  }
}

// (Z, ZT and, in pass 2, D are read through plain pointers: in the persistent
// batch kernel they are written earlier in the same launch, and a restricted
// pointer read at a wavefront-uniform index could be served from the scalar
// cache, which a device-scope acquire does not refresh.)
// N and D of v in closed form from k, As = sum k_a, Q = sum k_a^2 and
// A2 = sum asum[a] over the neighbours a (summing the per-arc identities
// N_e = (k-1) + (k_a-1) and
// D_e = (k-1)(k+k_a-4) + (As-k_a) + (k_a-1)(k_a+k-4) + (asum[a]-k)),
// less 8 per triangle.
template <typename T>
__device__ __forceinline__ void fin_store(int32_t v, int32_t k, int64_t As, longlong2 qa,
                                          bool has_z, typename SumT<T>::type sacc, double tfix,
                                          int64_t Tc, const void *Z,
                                          const int64_t *ZT, double *ef,
                                          int64_t *Dout, int64_t *Nout, uint8_t *fl) {
  using S = SumT<T>;
  typename S::type z = typename S::type();
  // Z, ZT: written by the triangle walk of nodes that have segments
  if (has_z) {
    S::add_stored(z, Z, v);
    Tc += ZT[v];
  }
  const double tri = tfix * (1.0 / kTriFix) + S::value(z);
  const double Stot = S::value(sacc) + 4.0 * tri;
  const int64_t kk = k;
  const int64_t Nn = kk * kk - 2 * kk + As;
  const int64_t Dd = kk * (kk - 4) * (kk - 2) + (3 * kk - 7) * As + qa.x + qa.y - kk * kk - 8 * Tc;
  ef[v] = finish_ef<T>(Nn, Dd, Stot, v, fl);
  Dout[v] = Dd;
  Nout[v] = Nn;
}

struct FinArgs {
  const int32_t *row_ptr, *deg;
  const int2 *adj2;
  const int32_t *rrev, *trec, *dn_ptr;  // rrev: where R holds each arc's reverse sum
  const int64_t *asum;
  const longlong2 *qa;
  const void *R;
  const TriSlot *Y;
  const void *Z;
  const int64_t *ZT;
  double *ef;
  int64_t *D, *N;
  uint8_t *fl;
};

// G lanes per node over `nodes` (NULL: node ids 0..count-1 of degree <= kmax),
// using blocks 0 .. nblk-1 of this role
template <typename T, int G>
__device__ __forceinline__ void fin_groups(const FinArgs &A, const int32_t *nodes, int64_t count,
                                           int32_t kmax, int64_t blk, int64_t nblk) {
  using Acc = typename SumT<T>::type;
  const int sub = threadIdx.x & (G - 1);
  const int64_t grp = (blk * blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = (nblk * blockDim.x) / G;
  // every lane of a wavefront runs the same number of rounds (group shuffles)
  const int64_t rounds = (count + ngrp - 1) / ngrp;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t it = r * ngrp + grp;
    int32_t v = -1, k = 0;
    if (it < count) {
      v = nodes ? nodes[it] : (int32_t)it;
      k = A.deg[v];
      if (!nodes && k > kmax) v = -1;
    }
    if (v < 0) k = 0;
    Acc sacc = Acc();
    double tfix = 0.0;
    int64_t Tc = 0;
    if (v >= 0)
      fin_arcs<T>(A.adj2, A.rrev, A.trec, A.R, A.Y, k, A.row_ptr[v], sub, G, sacc, tfix, Tc);
    sacc = group_sum<G>(sacc);
    tfix = group_sum<G>(tfix);
    Tc = group_sum<G>(Tc);
    if (v >= 0 && sub == 0)
      fin_store<T>(v, k, A.asum[v], A.qa[v], A.dn_ptr[v + 1] > A.dn_ptr[v], sacc, tfix, Tc, A.Z,
                   A.ZT, A.ef, A.D, A.N, A.fl);
  }
}

// one lane per node of degree <= kFinLaneMax over node ids 0..n-1: the loads
// of all of a node's arcs are issued together (indices clamped to its row,
// contributions past k masked), so a node costs two dependent round trips
template <typename T> struct RVal;
template <> struct RVal<float> {
  __device__ static float load(const void *R, int64_t i) {
    return reinterpret_cast<const float *>(R)[i];
  }
  __device__ static void add(DFv &a, float x, bool on) { a.add(on ? x : 0.0f); }
};
template <> struct RVal<double> {
  __device__ static double load(const void *R, int64_t i) {
    return reinterpret_cast<const double *>(R)[i];
  }
  __device__ static void add(double &a, double x, bool on) { a += on ? x : 0.0; }
};

template <typename T>
__device__ __forceinline__ void fin_lanes(const FinArgs &A, int64_t lo, int64_t hi, int64_t blk,
                                          int64_t nblk) {
  using Acc = typename SumT<T>::type;
  constexpr int K = kFinLaneMax;
  const int64_t stride = nblk * (int64_t)blockDim.x;
  for (int64_t v = lo + blk * (int64_t)blockDim.x + threadIdx.x; v < hi; v += stride) {
    const int32_t k = A.deg[v];
    if (k > K) continue;
    Acc sacc = Acc();
    double tfix = 0.0;
    int64_t Tc = 0;
    if (k > 0) {
      const int32_t base = A.row_ptr[v];
      int32_t ka[K], rv[K], tr[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int32_t e = base + (i < k ? i : k - 1);
        ka[i] = A.adj2[e].y;
        rv[i] = A.rrev[e];
        tr[i] = A.trec[e];
      }
      decltype(RVal<T>::load(A.R, 0)) own[K], back[K];
      TriSlot ts[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        own[i] = RVal<T>::load(A.R, base + (i < k ? i : k - 1));
        back[i] = RVal<T>::load(A.R, rv[i]);
        ts[i] = A.Y[tr[i] >= 0 ? tr[i] : 0];
      }
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const bool in = i < k;
        // a centre of degree 1 has no pairs: its row sums were never written
        RVal<T>::add(sacc, own[i], in && k >= 2);
        RVal<T>::add(sacc, back[i], in && ka[i] >= 2);
        const bool hit = in && tr[i] >= 0;
        tfix += hit ? (double)ts[i].y : 0.0;
        Tc += hit ? ts[i].t : 0;
      }
    }
    fin_store<T>((int32_t)v, k, A.asum[v], A.qa[v], A.dn_ptr[v + 1] > A.dn_ptr[v], sacc, tfix,
                 Tc, A.Z, A.ZT, A.ef, A.D, A.N, A.fl);
  }
}

// one workgroup (up to 16 wavefronts) per hub; partials combined in a fixed order
template <typename T>
__device__ __forceinline__ void fin_hubs(const FinArgs &A, const int32_t *nodes, int64_t count,
                                         int64_t blk, int64_t nblk) {
  using Acc = typename SumT<T>::type;
  __shared__ Acc shS[16];
  __shared__ double shT[16];
  __shared__ int64_t shC[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = (int)(blockDim.x >> 6);
  for (int64_t it = blk; it < count; it += nblk) {
    const int32_t v = nodes[it];
    const int32_t k = A.deg[v];
    Acc sacc = Acc();
    double tfix = 0.0;
    int64_t Tc = 0;
    fin_arcs<T>(A.adj2, A.rrev, A.trec, A.R, A.Y, k, A.row_ptr[v], tid, (int32_t)blockDim.x, sacc,
                tfix, Tc);
    sacc = wave_sum(sacc);
    tfix = wave_sum_f64(tfix);
    Tc = wave_sum_i64(Tc);
    if (lane == 0) {
      shS[wv] = sacc;
      shT[wv] = tfix;
      shC[wv] = Tc;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < nw; ++w) {
        acc_merge(sacc, shS[w]);
        tfix += shT[w];
        Tc += shC[w];
      }
      fin_store<T>(v, k, A.asum[v], A.qa[v], A.dn_ptr[v + 1] > A.dn_ptr[v], sacc, tfix, Tc, A.Z,
                   A.ZT, A.ef, A.D, A.N, A.fl);
    }
    __syncthreads();
  }
}

// One launch for every node: block ranges select the role, hubs first so
// their long rows overlap with the rest.
//   [0, b0)        hubs (degree > kFinBlockMin), a workgroup each
//   [b0, b1)       degree kFinHalfMax+1 .. kFinBlockMin, a wavefront each
//   [b1, b2)       degree kFinGroupMax+1 .. kFinHalfMax, 32 lanes each
//   [b2, b3)       degree kFinLaneMax+1 .. kFinGroupMax, 8 lanes each (list by id)
//   [b3, grid)     degree <= kFinLaneMax, one lane each (node ids)
template <typename T>
__global__ __launch_bounds__(256) void k_finalize_cluster(
    FinArgs A, const int32_t *l_hub, int64_t n_hub, const int32_t *l_wave, int64_t n_wave,
    const int32_t *l_half, int64_t n_half, const int32_t *l_group, int64_t n_group, int32_t n,
    int64_t b0, int64_t b1, int64_t b2, int64_t b3) {
  const int64_t b = blockIdx.x;
  if (b < b0) fin_hubs<T>(A, l_hub, n_hub, b, b0);
  else if (b < b1) fin_groups<T, 64>(A, l_wave, n_wave, 0, b - b0, b1 - b0);
  else if (b < b2) fin_groups<T, 32>(A, l_half, n_half, 0, b - b1, b2 - b1);
  else if (b < b3) fin_groups<T, 8>(A, l_group, n_group, 0, b - b2, b3 - b2);
  else fin_lanes<T>(A, 0, n, b - b3, (int64_t)gridDim.x - b3);
}

static unsigned cap_blocks(int64_t b, int64_t cap) {
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

hipError_t launch_finalize_cluster(const Graph &g, ef_prec prec, const void *R, const TriSlot *Y,
                                   const void *Z, const int64_t *ZT, double *ef, int64_t *D,
                                   int64_t *N, uint8_t *fl, hipStream_t st) {
  // fin_list = [hubs][wavefront tier][32-lane tier] (degree descending), then
  // the 8-lane tier (id order)
  const int64_t n_wave = g.n_fin - g.n_fin_hub - g.n_fin_half;
  const int32_t *l_wave = g.fin_list + g.n_fin_hub, *l_half = l_wave + n_wave;
  const int32_t *l_group = g.fin_list + g.n_fin;
  const int64_t bh = g.n_fin_hub > 0 ? cap_blocks(g.n_fin_hub, 1 << 14) : 0;
  const int64_t bw = n_wave > 0 ? cap_blocks((n_wave * 64 + 255) / 256, 1 << 18) : 0;
  const int64_t bc = g.n_fin_half > 0 ? cap_blocks((g.n_fin_half * 32 + 255) / 256, 1 << 18) : 0;
  const int64_t bg = g.n_fin_group > 0 ? cap_blocks((g.n_fin_group * 8 + 255) / 256, 1 << 18) : 0;
  const int64_t bl = cap_blocks(((int64_t)g.n + 255) / 256, 1 << 17);
  const FinArgs A{g.row_ptr, g.deg, g.adj2, g.rrev, g.trec, g.dn_ptr, g.asum, g.qa,
                  R,         Y,     Z,      ZT,    ef,     D,      N,        fl};
  const unsigned grid = (unsigned)(bh + bw + bc + bg + bl);
  if (prec == EF_PREC_FP64)
    hipLaunchKernelGGL(k_finalize_cluster<double>, dim3(grid), dim3(256), 0, st, A, g.fin_list,
                       g.n_fin_hub, l_wave, n_wave, l_half, g.n_fin_half, l_group, g.n_fin_group,
                       g.n, bh, bh + bw, bh + bw + bc, bh + bw + bc + bg);
  else
    hipLaunchKernelGGL(k_finalize_cluster<float>, dim3(grid), dim3(256), 0, st, A, g.fin_list,
                       g.n_fin_hub, l_wave, n_wave, l_half, g.n_fin_half, l_group, g.n_fin_group,
                       g.n, bh, bh + bw, bh + bw + bc, bh + bw + bc + bg);
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
// per-seed formulation (the original visit of each seed's own clusters):
//   stars a-s-b: the pair loop's row sums R over the seed's own arcs, plus the
//     triangle adjustment for adjacent a, b (found in the 2-hop walk);
//   paths s-a-b: the walk over the rows of every neighbour a, each entry
//     (b, k_b) one cluster of degree k_s + k_a + k_b - 4, less 2 if b ~ s.
// The rows of N(s) form one concatenated sequence ("segments"), walked 64
// entries per wavefront step; membership b in N(s) comes from an LDS hash
// (all but the largest seeds) or a device bitmap. N and D are exact integers.
// ---------------------------------------------------------------------------
__global__ void k_bitmap_set(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                             const int32_t *__restrict__ seeds, const int32_t *__restrict__ list,
                             int64_t n_big, uint32_t *__restrict__ bm, int64_t words, int set) {
  for (int64_t bi = blockIdx.x; bi < n_big; bi += gridDim.x) {
    const int32_t pos = list[bi];
    const int32_t s = seeds ? seeds[pos] : pos;
    uint32_t *b = bm + bi * words;
    for (int32_t e = row_ptr[s] + threadIdx.x; e < row_ptr[s + 1]; e += blockDim.x) {
      const int32_t x = col[e];
      if (set) atomicOr(&b[x >> 5], 1u << (x & 31));
      else b[x >> 5] = 0u;
    }
  }
}

// segment table of neighbours c0 .. c0+cnt-1 of a seed (row base `base`):
// seg[j] = {row start of a_j minus its first concatenated index, k_{a_j}},
// segp[j] = first concatenated index, segp[cnt] = total. NT threads.
template <int NT>
__device__ __forceinline__ int32_t seed_chunk_setup(const int32_t *__restrict__ row_ptr,
                                                    const int2 *__restrict__ adj2, int32_t base,
                                                    int32_t c0, int32_t cnt, int tid, int2 *seg,
                                                    int32_t *segp, int32_t *part) {
  int32_t run = 0;
  for (int32_t j0 = 0; j0 < cnt; j0 += NT) {
    const int32_t j = j0 + tid;
    int32_t a = 0, ka = 0;
    if (j < cnt) {
      const int2 ad = adj2[base + c0 + j];
      a = ad.x;
      ka = ad.y;
    }
    int32_t tot;
    const int32_t excl = group_excl_scan<NT>(ka, part, tot);
    if (j < cnt) {
      seg[j] = make_int2(row_ptr[a] - (run + excl), ka);
      segp[j] = run + excl;
    }
    run += tot;
  }
  if (tid == 0) segp[cnt] = run;
  return run;
}

template <int SLOTS>
__device__ __forceinline__ int32_t hash_insert(int32_t *hkey, int32_t x) {
  return LdsHash<SLOTS>::insert(hkey, x);
}

// one wavefront walks entries [beg, end) of the current chunk
template <typename T, int SLOTS, bool BITMAP>
__device__ __forceinline__ void seed_walk(const int2 *__restrict__ adj2, const int2 *seg,
                                          const int32_t *segp, int32_t nseg, int32_t beg,
                                          int32_t end, int32_t s, int32_t k, const int32_t *hkey,
                                          const uint32_t *__restrict__ bm, int32_t *flg,
                                          typename SumT<T>::type &sacc, int64_t &Dd,
                                          int64_t &Nn) {
  using S = SumT<T>;
  // per-round partials: at most 4 terms per lane, folded into the compensated
  // and 64-bit sums after each round (d < 3 * kMaxDegree, so 4 fit in int32)
  static_assert(4LL * 3 * kMaxDegree < (1LL << 31), "per-round degree sum overflows");
  T rs = T(0);
  int32_t rd = 0, rn = 0;
  seg_walk<4>(
      segp, nseg, beg, end, flg,
      [&](int32_t sg, int32_t idx) {
        const int2 sv = seg[sg];
        const int2 bd = adj2[sv.x + idx];
        return make_int3(bd.x, bd.y, sv.y);
      },
      [&](int32_t, int32_t, int3 e, bool ok) {
        const int32_t b = e.x;
        if (!ok || b == s) return;
        bool m;
        if constexpr (BITMAP) {
          m = (bm[b >> 5] >> (b & 31)) & 1u;
        } else {
          m = LdsHash<SLOTS>::find(hkey, b) >= 0;
        }
        // path s-a-b has degree sigma - 4, less 2 if b ~ s; then the star
        // (a, b) with a ~ b, which the pair loop scored with degree sigma - 4,
        // takes delta(sigma) = g(sigma - 6) - g(sigma - 4). Together, for a
        // member b: 2 g(sigma - 6) - g(sigma - 4); both logs on every lane
        // (no divergent branch).
        const int32_t sigma = k + e.z + e.y;
        const T sf = (T)sigma;  // exact: sigma < 2^24
        const T g4 = score_nn(sf - T(4)), g6 = score_nn(sf - T(6));
        rs += m ? T(2) * g6 - g4 : g4;
        rd += sigma - 4 - (m ? 4 : 0);
        rn += 1;
      },
      [&]() {
        S::add_term(sacc, rs);
        Dd += rd;
        Nn += rn;
        rs = T(0);
        rd = 0;
        rn = 0;
      });
}

template <typename T>
__device__ __forceinline__ void seed_finish(int32_t pos, int32_t k, int64_t As,
                                            typename SumT<T>::type sacc, int64_t Nn, int64_t Dd,
                                            double *ef, int64_t *Dout, int64_t *Nout,
                                            uint8_t *fl) {
  using S = SumT<T>;
  const int64_t kk = k;
  Nn += kk * (kk - 1);
  Dd += kk * (kk - 1) * (kk - 4) + 2 * (kk - 1) * As;
  ef[pos] = finish_ef<T>(Nn, Dd, S::value(sacc), pos, fl);
  Dout[pos] = Dd;
  Nout[pos] = Nn;
}

// seeds of degree <= MAXK: one wavefront per seed, WPB independent
// wavefronts per workgroup, each with its own LDS hash and segment table
template <typename T, int SLOTS, int MAXK, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_seed_wave(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ deg,
    const int2 *__restrict__ adj2, const int64_t *__restrict__ asum,
    const int32_t *__restrict__ seeds, const int32_t *__restrict__ list, int64_t count,
    const void *__restrict__ R, double *__restrict__ ef, int64_t *__restrict__ Dout,
    int64_t *__restrict__ Nout, uint8_t *__restrict__ fl) {
  using S = SumT<T>;
  using Acc = typename S::type;
  static_assert(MAXK <= 64, "one neighbour per lane");
  __shared__ __align__(16) int32_t hkey_s[WPB][SLOTS];
  __shared__ int2 seg_s[WPB][MAXK];
  __shared__ int32_t segp_s[WPB][MAXK + 1];
  __shared__ int32_t flg_s[WPB][kFlg];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t *hkey = hkey_s[wv];
  int32_t *flg = flg_s[wv];
  flg[lane] = 0;
  const int64_t nwaves = (int64_t)gridDim.x * WPB;
  // the hash is cleared once; afterwards each lane empties the one slot it
  // filled (k <= 64), so a low-degree seed does not pay for the whole table
  for (int i = lane; i < SLOTS; i += 64) hkey[i] = -1;
  for (int64_t it = (int64_t)blockIdx.x * WPB + wv; it < count; it += nwaves) {
    const int32_t pos = list[it];
    const int32_t s = seeds ? seeds[pos] : pos;
    const int32_t k = deg[s], base = row_ptr[s];
    wave_sync();
    Acc sacc = Acc();
    int64_t Dd = 0, Nn = 0;
    int32_t myslot = -1;
    if (lane < k) {
      myslot = hash_insert<SLOTS>(hkey, adj2[base + lane].x);
      if (k >= 2) S::add_arc(sacc, R, base + lane);
    }
    const int32_t total =
        seed_chunk_setup<64>(row_ptr, adj2, base, 0, k, lane, seg_s[wv], segp_s[wv], nullptr);
    wave_sync();
    seed_walk<T, SLOTS, false>(adj2, seg_s[wv], segp_s[wv], k, 0, total, s, k, hkey, nullptr, flg,
                               sacc, Dd, Nn);
    sacc = wave_sum(sacc);
    Dd = wave_sum_i64(Dd);
    Nn = wave_sum_i64(Nn);
    if (lane == 0)
      seed_finish<T>(pos, k, asum[s], sacc, Nn, Dd, ef, Dout, Nout, fl);
    if (myslot >= 0) hkey[myslot] = -1;
    wave_sync();
  }
}

// one workgroup of WPB wavefronts per seed; neighbours in chunks of MAXK,
// each wavefront walking a contiguous share of a chunk's sequence. BITMAP:
// membership from bm + slot * words, slot = index in the list.
// Minimum wavefronts per SIMD asked of the compiler for a per-seed bin: 8
// (64 VGPRs, a few spilled) for the 2048- and 8192-slot hashes, which then
// fit four 8-wavefront or two 16-wavefront workgroups on a compute unit. The
// 2-hop stream waits on memory, and the doubled occupancy outweighs the
// spills (at R-MAT scale 22: 174.6 -> 151.6 and 181.9 -> 114.6 ms). The
// bitmap bin gained nothing that way; the 16384-slot bin is held to one
// workgroup per CU by its LDS.
constexpr int seed_block_min_waves(int slots) { return slots == 2048 || slots == 8192 ? 8 : 1; }

template <typename T, int SLOTS, int MAXK, int WPB, bool BITMAP>
__global__ __launch_bounds__(64 * WPB, seed_block_min_waves(SLOTS)) void k_seed_block(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ deg,
    const int2 *__restrict__ adj2, const int64_t *__restrict__ asum,
    const int32_t *__restrict__ seeds, const int32_t *__restrict__ list, int64_t count,
    const void *__restrict__ R, const uint32_t *__restrict__ bm, int64_t words,
    double *__restrict__ ef, int64_t *__restrict__ Dout, int64_t *__restrict__ Nout,
    uint8_t *__restrict__ fl) {
  using S = SumT<T>;
  using Acc = typename S::type;
  constexpr int NT = 64 * WPB;
  __shared__ __align__(16) int32_t hkey[BITMAP ? 4 : SLOTS];
  __shared__ int2 seg[MAXK];
  __shared__ int32_t segp[MAXK + 1];
  __shared__ int32_t flg_s[WPB][kFlg];
  __shared__ int32_t part[WPB];
  __shared__ Acc shA[WPB];
  __shared__ int64_t shD[WPB], shN[WPB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int32_t *flg = flg_s[wv];
  flg[lane] = 0;
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t pos = list[it];
    const int32_t s = seeds ? seeds[pos] : pos;
    const int32_t k = deg[s], base = row_ptr[s];
    const uint32_t *mybm = BITMAP ? bm + it * words : nullptr;
    if constexpr (!BITMAP) {
      for (int i = tid; i < SLOTS; i += NT) hkey[i] = -1;
      __syncthreads();
    }
    Acc sacc = Acc();
    int64_t Dd = 0, Nn = 0;
    for (int32_t j = tid; j < k; j += NT) {
      if constexpr (!BITMAP) hash_insert<SLOTS>(hkey, adj2[base + j].x);
      if (k >= 2) S::add_arc(sacc, R, base + j);
    }
    for (int32_t c0 = 0; c0 < k; c0 += MAXK) {
      const int32_t cnt = min(MAXK, k - c0);
      const int32_t total = seed_chunk_setup<NT>(row_ptr, adj2, base, c0, cnt, tid, seg, segp, part);
      __syncthreads();
      const int32_t steps = (total + 63) >> 6;
      const int32_t beg = (int32_t)(((int64_t)steps * wv / WPB) << 6);
      const int32_t fin = (int32_t)(((int64_t)steps * (wv + 1) / WPB) << 6);
      seed_walk<T, SLOTS, BITMAP>(adj2, seg, segp, cnt, beg, fin < total ? fin : total, s, k, hkey,
                                  mybm, flg, sacc, Dd, Nn);
      __syncthreads();
    }
    sacc = wave_sum(sacc);
    Dd = wave_sum_i64(Dd);
    Nn = wave_sum_i64(Nn);
    if (lane == 0) {
      shA[wv] = sacc;
      shD[wv] = Dd;
      shN[wv] = Nn;
    }
    __syncthreads();
    if (tid == 0) {
      Acc a = shA[0];
      int64_t dsum = shD[0], nsum = shN[0];
      for (int w = 1; w < WPB; ++w) {
        acc_merge(a, shA[w]);
        dsum += shD[w];
        nsum += shN[w];
      }
      seed_finish<T>(pos, k, asum[s], a, nsum, dsum, ef, Dout, Nout, fl);
    }
    __syncthreads();
  }
}

// slots of the LDS hash set of N(s) per bin (bin 4 uses bitmaps); a set
// holds at most half its slots
constexpr int kSeedSlots[4] = {4 * kSeedBin0, 4 * kSeedBin1, 4 * kSeedBin2, 2 * kSeedBin3};
static_assert(kSeedSlots[0] >= 2 * kSeedBin0 && kSeedSlots[1] >= 2 * kSeedBin1 &&
                  kSeedSlots[2] >= 2 * kSeedBin2 && kSeedSlots[3] >= 2 * kSeedBin3,
              "per-seed hash sets must stay at most half full");

template <typename T>
static void per_seed_impl(const Graph &g, const int32_t *seeds, const int32_t *const *lists,
                          const int64_t *counts, const void *R, const uint32_t *bitmaps,
                          int64_t words, double *ef, int64_t *D, int64_t *N, uint8_t *fl,
                          hipStream_t st) {
  if (counts[0] > 0)
    hipLaunchKernelGGL((k_seed_wave<T, kSeedSlots[0], kSeedBin0, 4>),
                       dim3(cap_blocks((counts[0] + 3) / 4, 1 << 20)), dim3(256), 0, st,
                       g.row_ptr, g.deg, g.adj2, g.asum, seeds, lists[0], counts[0], R, ef, D, N,
                       fl);
  if (counts[1] > 0)
    hipLaunchKernelGGL((k_seed_block<T, kSeedSlots[1], kSeedBin1, 8, false>),
                       dim3(cap_blocks(counts[1], 1 << 20)), dim3(512), 0, st, g.row_ptr, g.deg,
                       g.adj2, g.asum, seeds, lists[1], counts[1], R, nullptr, words, ef, D, N,
                       fl);
  if (counts[2] > 0)
    hipLaunchKernelGGL((k_seed_block<T, kSeedSlots[2], kSeedChunk, 16, false>),
                       dim3(cap_blocks(counts[2], 1 << 20)), dim3(1024), 0, st, g.row_ptr,
                       g.deg, g.adj2, g.asum, seeds, lists[2], counts[2], R, nullptr, words, ef,
                       D, N, fl);
  if (counts[3] > 0)
    hipLaunchKernelGGL((k_seed_block<T, kSeedSlots[3], kSeedChunk, 16, false>),
                       dim3(cap_blocks(counts[3], 1 << 20)), dim3(1024), 0, st, g.row_ptr,
                       g.deg, g.adj2, g.asum, seeds, lists[3], counts[3], R, nullptr, words, ef,
                       D, N, fl);
  if (counts[4] > 0)
    hipLaunchKernelGGL((k_seed_block<T, 1, kSeedChunk, 16, true>),
                       dim3(cap_blocks(counts[4], 1 << 20)), dim3(1024), 0, st, g.row_ptr,
                       g.deg, g.adj2, g.asum, seeds, lists[4], counts[4], R, bitmaps, words, ef,
                       D, N, fl);
}

hipError_t launch_per_seed(const Graph &g, ef_prec prec, const int32_t *seeds,
                           const int32_t *const *lists, const int64_t *counts, const void *R,
                           uint32_t *bitmaps, double *ef, int64_t *D, int64_t *N, uint8_t *fl,
                           hipStream_t st, hipEvent_t ev_stream_done) {
  const int64_t words = ((int64_t)g.n + 31) / 32;
  constexpr int L = kSeedBins - 1;
  if (counts[L] > 0)
    hipLaunchKernelGGL(k_bitmap_set, dim3(cap_blocks(counts[L], 65536)), dim3(256), 0, st,
                       g.row_ptr, g.col_idx, seeds, lists[L], counts[L], bitmaps, words, 1);
  if (prec == EF_PREC_FP64)
    per_seed_impl<double>(g, seeds, lists, counts, R, bitmaps, words, ef, D, N, fl, st);
  else
    per_seed_impl<float>(g, seeds, lists, counts, R, bitmaps, words, ef, D, N, fl, st);
  if (ev_stream_done) (void)hipEventRecord(ev_stream_done, st);
  if (counts[L] > 0)
    hipLaunchKernelGGL(k_bitmap_set, dim3(cap_blocks(counts[L], 65536)), dim3(256), 0, st,
                       g.row_ptr, g.col_idx, seeds, lists[L], counts[L], bitmaps, words, 0);
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

// FP32C pass 2 of one flagged seed s (output position pos) on a workgroup
// (every thread calls it: it holds workgroup barriers). LDS: the seed's
// neighbours and their pairwise adjacency bits for k <= kP2Max.
struct Pass2Lds {
  int32_t nid[kP2Max], nk[kP2Max];
  uint32_t bits[kP2Max * (kP2Max / 32)];
  DFv sh[16];
};

__device__ __forceinline__ void pass2_seed(const int32_t *__restrict__ row_ptr,
                                           const int32_t *__restrict__ col,
                                           const int32_t *__restrict__ deg,
                                           const int2 *__restrict__ adj2, int32_t s, int32_t pos,
                                           double *ef, const int64_t *Dv, Pass2Lds &L) {
  const int tid = threadIdx.x, nt = (int)blockDim.x;
  const int32_t k = deg[s], base = row_ptr[s];
  const int64_t D = Dv[pos];
  const bool lds = k <= kP2Max;
  constexpr int W = kP2Max / 32;
  if (lds) {
    for (int i = tid; i < k; i += nt) {
      const int2 ad = adj2[base + i];
      L.nid[i] = ad.x;
      L.nk[i] = ad.y;
    }
    for (int i = tid; i < k * W; i += nt) L.bits[i] = 0u;
  }
  __syncthreads();
  DFv acc = DFv();
  // paths s -> a -> b (one event order each)
  for (int32_t i = 0; i < k; ++i) {
    const int2 ad = adj2[base + i];
    const int32_t a = ad.x, ka = ad.y;
    for (int32_t f = row_ptr[a] + tid; f < row_ptr[a + 1]; f += nt) {
      const int2 bd = adj2[f];
      const int32_t b = bd.x;
      if (b == s) continue;
      const int32_t j = lds ? find_sorted(L.nid, k, b) : find_sorted(col + base, k, b);
      if (j >= 0 && lds) atomicOr(&L.bits[i * W + (j >> 5)], 1u << (j & 31));
      acc.add(term_nonneg(k + ka + bd.y - 4 - (j >= 0 ? 2 : 0), D));
    }
  }
  __syncthreads();
  // stars a - s - b (two event orders each)
  for (int32_t i = 0; i < k; ++i) {
    const int32_t a = lds ? L.nid[i] : adj2[base + i].x;
    const int32_t ka = lds ? L.nk[i] : adj2[base + i].y;
    for (int32_t j = i + 1 + tid; j < k; j += nt) {
      const int32_t kb = lds ? L.nk[j] : adj2[base + j].y;
      bool m;
      if (lds) m = (L.bits[i * W + (j >> 5)] >> (j & 31)) & 1u;
      else m = find_sorted(col + row_ptr[a], deg[a], col[base + j]) >= 0;
      const float t = term_nonneg(k + ka + kb - 4 - (m ? 2 : 0), D);
      acc.add(t);
      acc.add(t);
    }
  }
  acc = block_sum_acc(acc, L.sh);
  if (tid == 0) {
    const double e = acc.value() / (double)D;
    ef[pos] = e > 0.0 ? e : 0.0;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_pass2(const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col,
                                               const int32_t *__restrict__ deg,
                                               const int2 *__restrict__ adj2,
                                               const int32_t *__restrict__ seeds,
                                               const int32_t *__restrict__ flagged,
                                               const int32_t *__restrict__ flag_count,
                                               double *__restrict__ ef,
                                               const int64_t *__restrict__ Dv) {
  __shared__ Pass2Lds L;
  const int32_t count = *flag_count;
  for (int32_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t pos = flagged[it];
    pass2_seed(row_ptr, col, deg, adj2, seeds ? seeds[pos] : pos, pos, ef, Dv, L);
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
