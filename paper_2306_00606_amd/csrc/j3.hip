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
// Decomposition. A work item is one first event s -> y (an arc of s). Its
// second events ("prefixes") are s -> z, z in N(s) \ {y}, and y -> z,
// z in N(y) \ {s}; a prefix leaves T = {s, y, z} with
// d_T = k_s + k_y + k_z - 2 e(T), e(T) = 2 + [z adjacent to the other of
// s, y]. Its third events are the edges leaving T: a node w outside T joined
// to c_w >= 1 members of T gives c_w events, each with
// d_J = d_T + k_w - 2 c_w. With the rows sorted by id, a three-way merge of
// N(s), N(y) and N(z) meets every such w exactly c_w times in a row, so one
// lane per prefix walks the merge and needs no set structure. The item's
// sums (event count, sum of d_J, sum of g(d_J)) are stored per arc and
// summed per seed.
//
// Precision: FP64 scores d ln d in double. FP32C scores d log2 d with
// v_log_f32, summed in double; the seed's EF is taken in double. Seeds whose
// EF cancels (kappa = (S/D) / EF > 16, or EF <= 0) are flagged, and the
// caller recomputes their items in FP64.
#include "common.cuh"

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

// Items: the arcs of seeds[0 .. nseeds), seed i owning items
// off[i] .. off[i+1] (its arcs in row order). One wavefront per item, one lane
// per prefix; the item's event count, degree sum and score sum go to
// PN / PD / PS at the arc's index.
template <typename T>
__global__ __launch_bounds__(256) void k_j3_items(const int32_t *__restrict__ row_ptr,
                                                  const int2 *__restrict__ adj2,
                                                  const int32_t *__restrict__ rev,
                                                  const int32_t *__restrict__ seeds,
                                                  const int64_t *__restrict__ off, int32_t nseeds,
                                                  long long *__restrict__ PN,
                                                  long long *__restrict__ PD,
                                                  double *__restrict__ PS) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t n_items = off[nseeds];
  for (int64_t it = wave; it < n_items; it += nwaves) {
    // seed of the item: the last i with off[i] <= it
    int32_t lo = 0, hi = nseeds;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (off[mid] <= it) lo = mid; else hi = mid;
    }
    const int32_t s = seeds[lo];
    const int32_t s0 = row_ptr[s], s1 = row_ptr[s + 1], ks = s1 - s0;
    const int32_t e = s0 + (int32_t)(it - off[lo]);
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

static unsigned j3_blocks(int64_t threads) {
  int64_t b = (threads + 255) / 256;
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (unsigned)b;
}

hipError_t launch_j3_items(const Graph &g, bool fp64, const int32_t *seeds, const int64_t *off,
                           int32_t nseeds, int64_t n_items, long long *PN, long long *PD,
                           double *PS, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  const unsigned blocks = j3_blocks(n_items * 64);
  if (fp64)
    hipLaunchKernelGGL(k_j3_items<double>, dim3(blocks), dim3(256), 0, st, g.row_ptr, g.adj2,
                       g.rev, seeds, off, nseeds, PN, PD, PS);
  else
    hipLaunchKernelGGL(k_j3_items<float>, dim3(blocks), dim3(256), 0, st, g.row_ptr, g.adj2,
                       g.rev, seeds, off, nseeds, PN, PD, PS);
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
