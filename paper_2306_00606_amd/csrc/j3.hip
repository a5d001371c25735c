// Expected Force with three transmission events (Sec. 3.3 defines EF for a
// number j of events; the paper uses j = 2).
//
// Sequences of seed s: event 1 s -> y; event 2 x2 -> z with x2 in {s, y};
// event 3 x3 -> w with x3 in {s, y, z}; every newly infected node is outside
// the infected set and adjacent to its infector. Each ordered sequence is one
// cluster instance, as Algorithm 1's multiplicities count them for j = 2. The
// cluster J = {s, y, z, w} has degree d_J = (sum of the four degrees) -
// 2 e(J). Then N = number of sequences, D = sum of d_J, S = sum of
// d_J ln d_J, and EF = ln D - S / D (Eq. 1).
//
// A work item is one first event s -> y (an arc of a seed). Its second events
// ("prefixes") are s -> z, z in N(s) \ {y}, and y -> z, z in N(y) \ {s}: one
// per entry of the list L = N(s) \ {y} ++ N(y) \ {s}. A prefix leaves
// T = {s, y, z} with d_T = k_s + k_y + k_z - 2 (1 + c_z), c_z the number of
// s, y adjacent to z. Its third events are the edges leaving T: a node w
// outside T joined to c_w members of T gives c_w events of degree
// d_T + k_w - 2 c_w; every prefix has d_T of them.
//
// Union path (k_j3_block): M = N(s) u N(y) \ {s, y}, with c_w in {1, 2} its
// adjacency to {s, y}, is hashed in LDS once per item and its entries held in
// registers. For a prefix, the nodes of M other than z give
//   A(d_T) = sum_{w in M} c_w g(d_T + k_w - 2 c_w)  less z's own term,
// evaluated for every prefix by a loop over the prefixes with their d_T read
// by broadcast; the neighbours of z then adjust: a w in M gains one edge into
// T, a w outside M adds one event of degree d_T + k_w - 2. Those are found
// by one segmented walk over the rows N(z) of all prefixes with hash
// lookups. The degree sum of the M part is a closed form per prefix.
// Merge path (k_j3_merge), for items whose list exceeds the largest hash: one
// lane per prefix walks a three-way merge of the sorted rows N(s), N(y),
// N(z), which meets every w exactly c_w times in a row.
// Item sums (event count, sum of d_J, sum of g(d_J)) are stored per arc and
// summed per seed.
//
// Precision: FP64 scores d ln d in double. FP32C scores d log2 d with
// v_log_f32 and sums them in double; the seed's EF is taken in double.
// Seeds whose EF cancels (kappa = (S/D) / EF > 16, or EF <= 0) are flagged,
// and the caller recomputes their items in FP64.
#include "device_common.h"

namespace efi {

constexpr int32_t kJ3End = 0x7FFFFFFF;  // past-the-end id of a merged row

// 1 if x is in the sorted row adj2[b .. e), else 0
__device__ __forceinline__ int32_t j3_in_row(const int2 *__restrict__ adj2, int32_t b, int32_t e,
                                             int32_t x) {
  const int32_t end = e;
  while (b < e) {
    const int32_t mid = (b + e) >> 1;
    if (adj2[mid].x < x) b = mid + 1; else e = mid;
  }
  return (b < end && adj2[b].x == x) ? 1 : 0;
}

__device__ __forceinline__ int2 j3_head(const int2 *__restrict__ adj2, int32_t i, int32_t e) {
  return i < e ? adj2[i] : make_int2(kJ3End, 0);
}

// g(d) summed in double: FP32C in log2 units, FP64 in natural log
template <typename T> __device__ __forceinline__ double j3_score(int32_t d);
template <> __device__ __forceinline__ double j3_score<float>(int32_t d) {
  return (double)score_t<float>(d);
}
template <> __device__ __forceinline__ double j3_score<double>(int32_t d) {
  return score_t<double>(d);
}

// Items of seeds[0 .. nseeds), seed i owning off[i] .. off[i+1] (its arcs in
// row order): the seed index of item it (the last i with off[i] <= it).
__device__ __forceinline__ int32_t j3_item_seed(const int64_t *__restrict__ off, int32_t nseeds,
                                                int64_t it) {
  int32_t lo = 0, hi = nseeds;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= it) lo = mid; else hi = mid;
  }
  return lo;
}

// Work bins by the list length L = k_s + k_y - 2 (prefixes, and a bound on
// |M|): the union kernel's hash holds up to kJ3Lmax[b] entries at load 1/2.
constexpr int kJ3Bins = 5;
constexpr int32_t kJ3LmaxW = 64, kJ3Lmax0 = 256, kJ3Lmax1 = 2048, kJ3Lmax2 = 8192;
__device__ __forceinline__ int j3_bin(int32_t L) {
  return L <= kJ3LmaxW ? 0 : L <= kJ3Lmax0 ? 1 : L <= kJ3Lmax1 ? 2 : L <= kJ3Lmax2 ? 3 : 4;
}

// Sort the items into per-bin lists of arcs (lists + b * cap), counts[b]
// advanced with one atomic per workgroup and bin (counts cleared before).
__global__ __launch_bounds__(256) void k_j3_bins(const int32_t *__restrict__ row_ptr,
                                                 const int2 *__restrict__ adj2,
                                                 const int32_t *__restrict__ seeds,
                                                 const int64_t *__restrict__ off, int32_t nseeds,
                                                 int32_t *__restrict__ lists, int64_t cap,
                                                 int32_t *__restrict__ counts) {
  __shared__ int32_t wcnt[4][kJ3Bins];
  __shared__ int32_t base[kJ3Bins];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t n_items = off[nseeds];
  for (int64_t b0 = (int64_t)blockIdx.x * 256; b0 < n_items; b0 += (int64_t)gridDim.x * 256) {
    const int64_t it = b0 + tid;
    int bin = -1;
    int32_t e = 0;
    if (it < n_items) {
      const int32_t i = j3_item_seed(off, nseeds, it);
      const int32_t sd = seeds[i];
      e = row_ptr[sd] + (int32_t)(it - off[i]);
      bin = j3_bin(row_ptr[sd + 1] - row_ptr[sd] + adj2[e].y - 2);
    }
    int32_t rank = 0;
    for (int b = 0; b < kJ3Bins; ++b) {
      const unsigned long long m = __ballot(bin == b);
      if (bin == b)
        rank = (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      if (lane == 0) wcnt[wv][b] = __popcll(m);
    }
    __syncthreads();
    if (tid < kJ3Bins) {
      const int32_t tot = wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
      static_assert(sizeof(wcnt) / sizeof(wcnt[0]) == 4, "four wavefronts per workgroup");
      base[tid] = tot ? atomicAdd(&counts[tid], tot) : 0;
    }
    __syncthreads();
    if (bin >= 0) {
      int32_t pre = 0;
      for (int w = 0; w < wv; ++w) pre += wcnt[w][bin];
      lists[bin * cap + base[bin] + pre + rank] = e;
    }
    __syncthreads();
  }
}

// Merge path: one wavefront per item (arc e of the list), one lane per prefix.
template <typename T>
__global__ __launch_bounds__(256) void k_j3_merge(const int32_t *__restrict__ row_ptr,
                                                  const int2 *__restrict__ adj2,
                                                  const int32_t *__restrict__ rev,
                                                  const int32_t *__restrict__ src,
                                                  const int32_t *__restrict__ items,
                                                  const int32_t *__restrict__ count_p,
                                                  long long *__restrict__ PN,
                                                  long long *__restrict__ PD,
                                                  double *__restrict__ PS) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t n_items = *count_p;
  for (int64_t it = wave; it < n_items; it += nwaves) {
    const int32_t e = items[it];
    const int32_t s = src[e];
    const int32_t s0 = row_ptr[s], s1 = row_ptr[s + 1], ks = s1 - s0;
    const int2 yk = adj2[e];
    const int32_t y = yk.x, ky = yk.y;
    const int32_t y0 = row_ptr[y], y1 = row_ptr[y + 1];
    const int32_t py = e - s0;        // position of y in N(s)
    const int32_t ps = rev[e] - y0;   // position of s in N(y)
    const int32_t P = (ks - 1) + (ky - 1);
    long long cn = 0, cd = 0;
    double cs = 0.0;
    for (int32_t p0 = 0; p0 < P; p0 += 64) {
      const int32_t p = p0 + lane;
      if (p >= P) continue;
      int2 zk;
      int32_t eT;
      if (p < ks - 1) {  // s -> z, z in N(s) \ {y}
        zk = adj2[s0 + p + (p >= py ? 1 : 0)];
        eT = 2 + j3_in_row(adj2, y0, y1, zk.x);
      } else {  // y -> z, z in N(y) \ {s}
        const int32_t q = p - (ks - 1);
        zk = adj2[y0 + q + (q >= ps ? 1 : 0)];
        eT = 2 + j3_in_row(adj2, s0, s1, zk.x);
      }
      const int32_t z = zk.x;
      const int32_t dT = ks + ky + zk.y - 2 * eT;
      const int32_t z0 = row_ptr[z], z1 = row_ptr[z + 1];
      int32_t ia = s0, ib = y0, ic = z0;
      int2 a = j3_head(adj2, ia, s1), b = j3_head(adj2, ib, y1), c = j3_head(adj2, ic, z1);
      for (;;) {
        const int32_t w = min(a.x, min(b.x, c.x));
        if (w == kJ3End) break;
        const bool ma = a.x == w, mb = b.x == w, mc = c.x == w;
        const int32_t cw = (int32_t)ma + (int32_t)mb + (int32_t)mc;
        const int32_t kw = ma ? a.y : (mb ? b.y : c.y);
        if (w != s && w != y && w != z) {
          const int32_t d = dT + kw - 2 * cw;
          cn += cw;
          cd += (long long)cw * d;
          cs += (double)cw * j3_score<T>(d);
        }
        if (ma) a = j3_head(adj2, ++ia, s1);
        if (mb) b = j3_head(adj2, ++ib, y1);
        if (mc) c = j3_head(adj2, ++ic, z1);
      }
    }
    cn = wave_sum_i64(cn);
    cd = wave_sum_i64(cd);
    cs = wave_sum_f64(cs);
    if (lane == 0) {
      PN[e] = cn;
      PD[e] = cd;
      PS[e] = cs;
    }
  }
}

// Slot of key x in an LDS table of DS slots (power of two, at most half
// full), inserting it when absent.
template <int DS>
__device__ __forceinline__ int32_t j3_find_or_insert(int32_t *keys, int32_t x) {
  uint32_t h = ((uint32_t)x * 0x9E3779B1u) >> (32 - __builtin_ctz(DS));
  for (;;) {
    const int32_t old = atomicCAS(&keys[h], -1, x);
    if (old == -1 || old == x) return (int32_t)h;
    h = (h + 1) & (DS - 1);
  }
}

// Union path: one workgroup of WPB wavefronts per item (arc e of the list,
// list length L <= SLOTS / 2), prefixes in chunks of PCH. Within a chunk the
// M part depends on a prefix only through d_T: it is evaluated once per
// distinct d_T and weighted by the number of prefixes that share it.
template <typename T> struct J3Acc;
template <> struct J3Acc<float> {
  using type = float;
  __device__ static float g(int32_t d) { return score_t<float>(d); }
};
template <> struct J3Acc<double> {
  using type = double;
  __device__ static double g(int32_t d) { return score_t<double>(d); }
};

template <typename T, int SLOTS, int WPB, int PCH>
__global__ __launch_bounds__(64 * WPB) void k_j3_block(const int32_t *__restrict__ row_ptr,
                                                        const int2 *__restrict__ adj2,
                                                        const int32_t *__restrict__ rev,
                                                        const int32_t *__restrict__ src,
                                                        const int32_t *__restrict__ items,
                                                        const int32_t *__restrict__ count_p,
                                                        long long *__restrict__ PN,
                                                        long long *__restrict__ PD,
                                                        double *__restrict__ PS) {
  constexpr int NT = 64 * WPB;
  constexpr int LMAX = SLOTS / 2;
  constexpr int MR = (LMAX + NT - 1) / NT;  // list entries per thread
  static_assert(PCH % NT == 0 && LMAX % PCH == 0, "chunks of whole thread rounds");
  using G = J3Acc<T>;
  using V = typename G::type;
  __shared__ __align__(16) int32_t hkey[SLOTS];
  __shared__ uint8_t hc[SLOTS];
  __shared__ int2 seg[PCH];  // {first index of z's row minus its concatenated start, d_T}
  __shared__ int32_t segp[PCH + 1];
  constexpr int DS = 2 * PCH;  // distinct d_T of a chunk: value -> count
  __shared__ int32_t dkey[DS];
  __shared__ int32_t dcnt[DS];
  __shared__ int2 uniq[PCH];  // {d_T, number of prefixes}
  __shared__ int32_t flg_s[WPB][kFlg];
  __shared__ int32_t part[WPB];
  __shared__ long long red_a[WPB], red_b[WPB];
  __shared__ double red_c[WPB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int32_t *flg = flg_s[wv];
  flg[lane] = 0;
  for (int i = tid; i < SLOTS; i += NT) hkey[i] = -1;
  for (int i = tid; i < DS; i += NT) {
    dkey[i] = -1;
    dcnt[i] = 0;
  }
  __syncthreads();
  const int64_t n_items = *count_p;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int32_t e = items[it];
    const int32_t s = src[e];
    const int32_t s0 = row_ptr[s], ks = row_ptr[s + 1] - s0;
    const int2 yk = adj2[e];
    const int32_t y = yk.x, ky = yk.y;
    const int32_t y0 = row_ptr[y];
    const int32_t py = e - s0, ps = rev[e] - y0;
    const int32_t L = ks + ky - 2;
    // the list entries of this thread: index tid + r NT
    int32_t zid[MR], kz[MR], slot[MR], cz[MR];
    bool dup[MR];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
      const int32_t i = tid + r * NT;
      slot[r] = -1;
      dup[r] = false;
      zid[r] = 0;
      kz[r] = 0;
      if (i < ks - 1) {  // N(s) \ {y}
        const int2 w = adj2[s0 + i + (i >= py ? 1 : 0)];
        zid[r] = w.x;
        kz[r] = w.y;
        slot[r] = LdsHash<SLOTS>::insert(hkey, w.x);
        hc[slot[r]] = 1;
      } else if (i < L) {  // N(y) \ {s}
        const int32_t q = i - (ks - 1);
        const int2 w = adj2[y0 + q + (q >= ps ? 1 : 0)];
        zid[r] = w.x;
        kz[r] = w.y;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < MR; ++r) {
      const int32_t i = tid + r * NT;
      if (i >= ks - 1 && i < L) {
        const int32_t f = LdsHash<SLOTS>::find(hkey, zid[r]);
        if (f >= 0) {
          hc[f] = 2;  // in both rows: the N(s) entry carries it
          dup[r] = true;
        } else {
          slot[r] = LdsHash<SLOTS>::insert(hkey, zid[r]);
          hc[slot[r]] = 1;
        }
      }
    }
    __syncthreads();
    // multiplicities, M sums for the closed-form degree sums
    long long m1 = 0, m2 = 0;
#pragma unroll
    for (int r = 0; r < MR; ++r) {
      const int32_t i = tid + r * NT;
      cz[r] = 0;
      if (i < L) {
        cz[r] = dup[r] ? 2 : (int32_t)hc[slot[r]];
        if (!dup[r]) {
          m1 += cz[r];
          m2 += (long long)cz[r] * (kz[r] - 2 * cz[r]);
        }
      }
    }
    m1 = wave_sum_i64(m1);
    m2 = wave_sum_i64(m2);
    if (lane == 0) {
      red_a[wv] = m1;
      red_b[wv] = m2;
    }
    __syncthreads();
    long long M1 = 0, M2 = 0;
    for (int w = 0; w < WPB; ++w) {
      M1 += red_a[w];
      M2 += red_b[w];
    }
    // per prefix (its owner thread): event count d_T, the M part's degree
    // sum, and z's own term, which the M loop below includes
    long long cn = 0, cd = 0;
    double cs = 0.0;
    int32_t dT[MR];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
      const int32_t i = tid + r * NT;
      dT[r] = 0;
      if (i < L) {
        const int32_t c = cz[r];
        dT[r] = ks + ky + kz[r] - 2 * (1 + c);
        cn += dT[r];
        cd += (long long)dT[r] * (M1 - c) + M2 - (long long)c * (kz[r] - 2 * c);
        cs -= (double)c * (double)G::g(dT[r] + kz[r] - 2 * c);
      }
    }
    // rounds of list entries this item uses (uniform)
    const int32_t rmax = (L + NT - 1) / NT;
    // M entries of this thread: weight c_w (0 for the second copy), k_w - 2 c_w
    V wgt[MR];
    int32_t kap[MR];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
      wgt[r] = (tid + r * NT < L && !dup[r]) ? (V)cz[r] : (V)0;
      kap[r] = kz[r] - 2 * cz[r];
    }
    for (int32_t p0 = 0; p0 < L; p0 += PCH) {
      const int32_t nseg = L - p0 < PCH ? L - p0 : PCH;
      // segment table of the chunk, in prefix order
      int32_t run = 0;
#pragma unroll
      for (int rr = 0; rr < PCH / NT; ++rr) {
        const int r = p0 / NT + rr;
        const int32_t i = tid + r * NT, j = i - p0;
        int32_t len = 0, zr = 0, d = 0;
#pragma unroll
        for (int q = 0; q < MR; ++q)
          if (q == r) {
            len = i < L ? kz[q] : 0;
            zr = zid[q];
            d = dT[q];
          }
        int32_t tot;
        const int32_t start = run + group_excl_scan<NT>(len, part, tot);
        if (i < L) {
          seg[j] = make_int2(row_ptr[zr] - start, d);
          segp[j] = start;
          atomicAdd(&dcnt[j3_find_or_insert<DS>(dkey, d)], 1);  // d_T >= 0
        }
        run += tot;
      }
      if (tid == 0) segp[nseg] = run;
      __syncthreads();
      // distinct d_T of the chunk, compacted in slot order (the table is
      // emptied on the way)
      int32_t nuniq = 0;
#pragma unroll
      for (int rr = 0; rr < DS / NT; ++rr) {
        const int32_t sl = tid + rr * NT;
        const int32_t key = dkey[sl], c = dcnt[sl];
        int32_t tot;
        const int32_t at = nuniq + group_excl_scan<NT>(key >= 0 ? 1 : 0, part, tot);
        if (key >= 0) {
          uniq[at] = make_int2(key, c);
          dkey[sl] = -1;
          dcnt[sl] = 0;
        }
        nuniq += tot;
      }
      __syncthreads();
      // M part: every distinct d_T against this thread's M entries
      for (int32_t u = 0; u < nuniq; ++u) {
        const int2 dc = uniq[u];
        V acc = 0;
#pragma unroll
        for (int r = 0; r < MR; ++r)
          if (r < rmax) acc += wgt[r] * G::g(dc.x + kap[r]);
        cs += (double)dc.y * (double)acc;
      }
      // z's neighbours: one walk over the chunk's rows N(z), wavefronts
      // taking contiguous shares
      const int32_t steps = (run + 63) >> 6;
      const int32_t beg = (int32_t)(((int64_t)steps * wv / WPB) << 6);
      const int32_t fin = (int32_t)(((int64_t)steps * (wv + 1) / WPB) << 6);
      seg_walk<4>(
          segp, nseg, beg, fin < run ? fin : run, flg,
          [&](int32_t sg, int32_t idx) { return adj2[seg[sg].x + idx]; },
          [&](int32_t sg, int32_t, int2 w, bool ok) {
            if (!ok || w.x == s || w.x == y) return;
            const int32_t d = seg[sg].y;
            const int32_t f = LdsHash<SLOTS>::find(hkey, w.x);
            if (f >= 0) {
              const int32_t c = hc[f];
              cs += (double)((c + 1) * G::g(d + w.y - 2 * c - 2) - c * G::g(d + w.y - 2 * c));
              cd += d + w.y - 4 * c - 2;
            } else {
              cs += (double)G::g(d + w.y - 2);
              cd += d + w.y - 2;
            }
          });
      __syncthreads();
    }
    cn = wave_sum_i64(cn);
    cd = wave_sum_i64(cd);
    cs = wave_sum_f64(cs);
    if (lane == 0) {
      red_a[wv] = cn;
      red_b[wv] = cd;
      red_c[wv] = cs;
    }
    __syncthreads();
    if (tid == 0) {
      long long a = 0, b = 0;
      double c = 0.0;
      for (int w = 0; w < WPB; ++w) {
        a += red_a[w];
        b += red_b[w];
        c += red_c[w];
      }
      PN[e] = a;
      PD[e] = b;
      PS[e] = c;
    }
    // empty the hash slots this thread filled
#pragma unroll
    for (int r = 0; r < MR; ++r)
      if (slot[r] >= 0) hkey[slot[r]] = -1;
    __syncthreads();
  }
}

// Per output position i (of `count`, or of the listed positions): node
// nodes[i] (i itself when nodes is null); N, D, S summed over the node's arcs
// and Eq. 1. FP32C flags (fl[i] = 1) positions whose EF cancels.
template <typename T>
__global__ __launch_bounds__(256) void k_j3_finish(const int32_t *__restrict__ row_ptr,
                                                   const long long *__restrict__ PN,
                                                   const long long *__restrict__ PD,
                                                   const double *__restrict__ PS,
                                                   const int32_t *__restrict__ nodes,
                                                   const int32_t *__restrict__ pos,
                                                   int32_t count, double *__restrict__ ef,
                                                   int64_t *__restrict__ Dout,
                                                   int64_t *__restrict__ Nout,
                                                   uint8_t *__restrict__ fl) {
  constexpr int G = 16;
  const int sub = threadIdx.x & (G - 1);
  const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
  const int64_t rounds = (count + ngrp - 1) / ngrp;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t t = r * ngrp + grp;
    int32_t i = -1, v = 0;
    if (t < count) {
      i = pos ? pos[t] : (int32_t)t;
      v = nodes ? nodes[i] : i;
    }
    long long n = 0, d = 0;
    double sc = 0.0;
    if (i >= 0)
      for (int32_t e = row_ptr[v] + sub; e < row_ptr[v + 1]; e += G) {
        n += PN[e];
        d += PD[e];
        sc += PS[e];
      }
    for (int o = G / 2; o > 0; o >>= 1) {
      n += __shfl_xor(n, o, G);
      d += __shfl_xor(d, o, G);
      sc += __shfl_xor(sc, o, G);
    }
    if (i < 0 || sub != 0) continue;
    double e1 = 0.0;
    uint8_t flag = 0;
    if (d > 0 && n > 1) {
      const double Dd = (double)d;
      const double sd = (sizeof(T) == 4 ? sc * 0.69314718055994530942 : sc) / Dd;
      e1 = log(Dd) - sd;
      if (sizeof(T) == 4 && (e1 <= 0.0 || sd > 16.0 * e1)) flag = 1;
      if (e1 <= 0.0) e1 = 0.0;  // never -0.0
    }
    ef[i] = e1;
    Dout[i] = d;
    Nout[i] = n;
    if (fl) fl[i] = flag;
  }
}

// Union path for short lists (L <= 64): one wavefront per item, one list
// entry (M entry and prefix) per lane, WPB wavefronts per workgroup with
// their own LDS state.
template <typename T, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_j3_wave(const int32_t *__restrict__ row_ptr,
                                                       const int2 *__restrict__ adj2,
                                                       const int32_t *__restrict__ rev,
                                                       const int32_t *__restrict__ src,
                                                       const int32_t *__restrict__ items,
                                                       const int32_t *__restrict__ count_p,
                                                       long long *__restrict__ PN,
                                                       long long *__restrict__ PD,
                                                       double *__restrict__ PS) {
  constexpr int SL = 2 * kJ3LmaxW;
  using G = J3Acc<T>;
  using V = typename G::type;
  __shared__ __align__(16) int32_t hkey_s[WPB][SL];
  __shared__ uint8_t hc_s[WPB][SL];
  __shared__ int2 seg_s[WPB][kJ3LmaxW];
  __shared__ int32_t segp_s[WPB][kJ3LmaxW + 1];
  __shared__ int32_t flg_s[WPB][kFlg];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t *hkey = hkey_s[wv], *segp = segp_s[wv], *flg = flg_s[wv];
  uint8_t *hc = hc_s[wv];
  int2 *seg = seg_s[wv];
  for (int i = lane; i < SL; i += 64) hkey[i] = -1;
  flg[lane] = 0;
  const int64_t nwaves = (int64_t)gridDim.x * WPB;
  const int64_t n_items = *count_p;
  for (int64_t it = (int64_t)blockIdx.x * WPB + wv; it < n_items; it += nwaves) {
    const int32_t e = items[it];
    const int32_t s = src[e];
    const int32_t s0 = row_ptr[s], ks = row_ptr[s + 1] - s0;
    const int2 yk = adj2[e];
    const int32_t y = yk.x, ky = yk.y;
    const int32_t y0 = row_ptr[y];
    const int32_t py = e - s0, ps = rev[e] - y0;
    const int32_t L = ks + ky - 2;
    const int32_t i = lane;
    int32_t zid = 0, kz = 0, slot = -1;
    bool dup = false;
    wave_sync();
    if (i < ks - 1) {  // N(s) \ {y}
      const int2 w = adj2[s0 + i + (i >= py ? 1 : 0)];
      zid = w.x;
      kz = w.y;
      slot = LdsHash<SL>::insert(hkey, w.x);
      hc[slot] = 1;
    } else if (i < L) {  // N(y) \ {s}
      const int32_t q = i - (ks - 1);
      const int2 w = adj2[y0 + q + (q >= ps ? 1 : 0)];
      zid = w.x;
      kz = w.y;
    }
    wave_sync();
    if (i >= ks - 1 && i < L) {
      const int32_t f = LdsHash<SL>::find(hkey, zid);
      if (f >= 0) {
        hc[f] = 2;
        dup = true;
      } else {
        slot = LdsHash<SL>::insert(hkey, zid);
        hc[slot] = 1;
      }
    }
    wave_sync();
    const int32_t c = i < L ? (dup ? 2 : (int32_t)hc[slot]) : 0;
    const long long M1 = wave_sum_i64(i < L && !dup ? c : 0);
    const long long M2 = wave_sum_i64(i < L && !dup ? (long long)c * (kz - 2 * c) : 0);
    const int32_t dT = i < L ? ks + ky + kz - 2 * (1 + c) : 0;
    long long cn = dT, cd = 0;
    double cs = 0.0;
    if (i < L) {
      cd = (long long)dT * (M1 - c) + M2 - (long long)c * (kz - 2 * c);
      cs = -(double)c * (double)G::g(dT + kz - 2 * c);
    }
    // M part: every prefix's d_T (read from its lane) against this lane's entry
    const V wgt = (i < L && !dup) ? (V)c : (V)0;
    const int32_t kap = kz - 2 * c;
    for (int32_t j = 0; j < L; ++j) {
      const int32_t d = __builtin_amdgcn_readlane(dT, j);
      cs += (double)(wgt * G::g(d + kap));
    }
    // segments: the rows N(z) of the prefixes
    int32_t tot = 0;
    {
      const int32_t len = i < L ? kz : 0;
      int32_t incl = len;
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
      }
      tot = __shfl(incl, 63, 64);
      const int32_t start = incl - len;
      if (i < L) {
        seg[i] = make_int2(row_ptr[zid] - start, dT);
        segp[i] = start;
      }
      if (lane == 0) segp[L] = tot;
    }
    wave_sync();
    seg_walk<4>(
        segp, L, 0, tot, flg, [&](int32_t sg, int32_t idx) { return adj2[seg[sg].x + idx]; },
        [&](int32_t sg, int32_t, int2 w, bool ok) {
          if (!ok || w.x == s || w.x == y) return;
          const int32_t d = seg[sg].y;
          const int32_t f = LdsHash<SL>::find(hkey, w.x);
          if (f >= 0) {
            const int32_t cw = hc[f];
            cs += (double)((cw + 1) * G::g(d + w.y - 2 * cw - 2) - cw * G::g(d + w.y - 2 * cw));
            cd += d + w.y - 4 * cw - 2;
          } else {
            cs += (double)G::g(d + w.y - 2);
            cd += d + w.y - 2;
          }
        });
    cn = wave_sum_i64(cn);
    cd = wave_sum_i64(cd);
    cs = wave_sum_f64(cs);
    if (lane == 0) {
      PN[e] = cn;
      PD[e] = cd;
      PS[e] = cs;
    }
    if (slot >= 0) hkey[slot] = -1;
  }
}

static unsigned j3_blocks(int64_t threads) {
  int64_t b = (threads + 255) / 256;
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (unsigned)b;
}

// The items of seeds[0 .. nseeds) (off: item offsets), binned by list length,
// each bin run by its kernel; lists: kJ3Bins * n_items ints, counts: kJ3Bins.
static_assert(kJ3Bins == 5, "list and count scratch sized for five bins");
hipError_t launch_j3_items(const Graph &g, bool fp64, const int32_t *seeds, const int64_t *off,
                           int32_t nseeds, int64_t n_items, int32_t *lists, int32_t *counts,
                           long long *PN, long long *PD, double *PS, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipError_t e = launch_zero_i32(counts, kJ3Bins, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_j3_bins, dim3(j3_blocks(n_items)), dim3(256), 0, st, g.row_ptr, g.adj2,
                     seeds, off, nseeds, lists, n_items, counts);
  const int32_t *l[kJ3Bins];
  for (int b = 0; b < kJ3Bins; ++b) l[b] = lists + b * n_items;
  if (fp64) {
    hipLaunchKernelGGL((k_j3_wave<double, 4>), dim3(8192), dim3(256), 0, st, g.row_ptr, g.adj2,
                       g.rev, g.src, l[0], counts + 0, PN, PD, PS);
    hipLaunchKernelGGL((k_j3_block<double, 2 * kJ3Lmax0, 4, 256>), dim3(4096), dim3(256), 0, st,
                       g.row_ptr, g.adj2, g.rev, g.src, l[1], counts + 1, PN, PD, PS);
    hipLaunchKernelGGL((k_j3_block<double, 2 * kJ3Lmax1, 8, 1024>), dim3(1024), dim3(512), 0, st,
                       g.row_ptr, g.adj2, g.rev, g.src, l[2], counts + 2, PN, PD, PS);
    hipLaunchKernelGGL((k_j3_block<double, 2 * kJ3Lmax2, 8, 1024>), dim3(256), dim3(512), 0, st,
                       g.row_ptr, g.adj2, g.rev, g.src, l[3], counts + 3, PN, PD, PS);
    hipLaunchKernelGGL(k_j3_merge<double>, dim3(2048), dim3(256), 0, st, g.row_ptr, g.adj2,
                       g.rev, g.src, l[4], counts + 4, PN, PD, PS);
  } else {
    hipLaunchKernelGGL((k_j3_wave<float, 4>), dim3(8192), dim3(256), 0, st, g.row_ptr, g.adj2,
                       g.rev, g.src, l[0], counts + 0, PN, PD, PS);
    hipLaunchKernelGGL((k_j3_block<float, 2 * kJ3Lmax0, 4, 256>), dim3(4096), dim3(256), 0, st,
                       g.row_ptr, g.adj2, g.rev, g.src, l[1], counts + 1, PN, PD, PS);
    hipLaunchKernelGGL((k_j3_block<float, 2 * kJ3Lmax1, 8, 1024>), dim3(1024), dim3(512), 0, st,
                       g.row_ptr, g.adj2, g.rev, g.src, l[2], counts + 2, PN, PD, PS);
    hipLaunchKernelGGL((k_j3_block<float, 2 * kJ3Lmax2, 8, 1024>), dim3(256), dim3(512), 0, st,
                       g.row_ptr, g.adj2, g.rev, g.src, l[3], counts + 3, PN, PD, PS);
    hipLaunchKernelGGL(k_j3_merge<float>, dim3(2048), dim3(256), 0, st, g.row_ptr, g.adj2,
                       g.rev, g.src, l[4], counts + 4, PN, PD, PS);
  }
  return hipGetLastError();
}

hipError_t launch_j3_finish(const Graph &g, bool fp64, const long long *PN, const long long *PD,
                            const double *PS, const int32_t *nodes, const int32_t *pos,
                            int32_t count, double *ef, int64_t *D, int64_t *N, uint8_t *fl,
                            hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const unsigned blocks = j3_blocks((int64_t)count * 16);
  if (fp64)
    hipLaunchKernelGGL(k_j3_finish<double>, dim3(blocks), dim3(256), 0, st, g.row_ptr, PN, PD,
                       PS, nodes, pos, count, ef, D, N, fl);
  else
    hipLaunchKernelGGL(k_j3_finish<float>, dim3(blocks), dim3(256), 0, st, g.row_ptr, PN, PD,
                       PS, nodes, pos, count, ef, D, N, fl);
  return hipGetLastError();
}

}  // namespace efi
