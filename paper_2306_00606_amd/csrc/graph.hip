// Graph preprocessing on the device: degrees, arc sources, reverse arcs, the
// packed (id, degree) adjacency, neighbour-degree sums and the
// degree-oriented half adjacency used by the triangle pass.
//
// The orientation ranks nodes by (degree, id): rank(a) < rank(b) when
// k_a < k_b, or k_a == k_b and a < b. up(u) = {w in N(u) : rank(w) > rank(u)}
// keeps every undirected edge exactly once and bounds |up(u)| by
// sqrt(2 * edges), which keeps the triangle pass short on skewed graphs.
// Each up(u) is stored in rank order, so the part of up(u) ranked above one
// of its members w is the contiguous tail after w. The triangle pass lists a
// triangle u < w < x at its middle node w, walking for every lower neighbour
// u of w that tail of up(u) against up(w); the per-node lists of those tails
// ("segments": slot of {u, w} in up(u), tail length, k_u + k_w) are built
// here, and every arc gets the index of the triangle record that holds the
// credits to its source node (-1 when no walk writes one).
#include <hipcub/hipcub.hpp>

#include "ef_internal.h"

namespace efi {

__device__ __forceinline__ bool rank_less(int32_t a, int32_t ka, int32_t b, int32_t kb) {
  return ka < kb || (ka == kb && a < b);
}

// flag[0] = 1 when a neighbour id lies outside [0, n); launch_check_cols
// clears the flag first
__global__ void k_check_clear(int32_t *__restrict__ flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

__global__ void k_check_cols(const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                             int32_t *__restrict__ flag) {
  bool bad = false;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    bad |= (uint32_t)col[e] >= (uint32_t)n;
  // one store per wavefront that saw a bad id
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_check_cols(const int32_t *col, int64_t nnz, int32_t n, int32_t *flag,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_check_clear, dim3(1), dim3(64), 0, st, flag);
  if (nnz > 0) {
    int64_t blocks = (nnz + 1023) / 1024;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_check_cols, dim3((unsigned)blocks), dim3(256), 0, st, col, nnz, n, flag);
  }
  return hipGetLastError();
}

__global__ void k_degree(const int32_t *__restrict__ row_ptr, int32_t n,
                         int32_t *__restrict__ deg) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    deg[v] = row_ptr[v + 1] - row_ptr[v];
}

// src[e] = the row that holds arc e (binary search over row_ptr).
__global__ void k_arc_src(const int32_t *__restrict__ row_ptr, int32_t n, int64_t nnz,
                          int32_t *__restrict__ src) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = n;  // find largest v with row_ptr[v] <= e
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) >> 1;
      if (row_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    src[e] = lo;
  }
}

__global__ void k_arc_rev(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                          const int32_t *__restrict__ src, const int32_t *__restrict__ deg,
                          int64_t nnz, int32_t *__restrict__ rev, int2 *__restrict__ adj2,
                          int32_t *__restrict__ upflag) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = src[e], a = col[e];
    int32_t lo = row_ptr[a], hi = row_ptr[a + 1];  // first position with col >= s
    while (lo < hi) {
      int32_t mid = (lo + hi) >> 1;
      if (col[mid] < s) lo = mid + 1; else hi = mid;
    }
    // on a valid (symmetric) graph the reverse arc is always found; keep the
    // index inside the row otherwise
    rev[e] = (lo < row_ptr[a + 1] && col[lo] == s) ? lo : (int32_t)e;
    const int32_t ka = deg[a];
    adj2[e] = make_int2(a, ka);
    upflag[e] = rank_less(s, deg[s], a, ka) ? 1 : 0;
  }
}

__global__ void k_up_fill(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                          const int32_t *__restrict__ rev, const int32_t *__restrict__ upflag,
                          const int32_t *__restrict__ upidx, int32_t n, int64_t nnz,
                          int32_t *__restrict__ up_ptr, int32_t *__restrict__ up_col,
                          int32_t *__restrict__ tslot) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride) {
    if (upflag[e]) {
      up_col[upidx[e]] = col[e];
      tslot[e] = upidx[e];
    } else {
      tslot[e] = upidx[rev[e]];
    }
  }
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += stride) {
    if (v < n) up_ptr[v] = (row_ptr[v] < nnz) ? upidx[row_ptr[v]] : (int32_t)(nnz / 2);
    else up_ptr[v] = (int32_t)(nnz / 2);
  }
}

// ---------------------------------------------------------------------------
// Rank order inside every up(u) (rows are in id order after k_up_fill).
// ---------------------------------------------------------------------------
__global__ void k_up_keys(const int32_t *__restrict__ up_col, const int32_t *__restrict__ deg,
                          int64_t nup, int32_t *__restrict__ upk) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nup;
       s += (int64_t)gridDim.x * blockDim.x)
    upk[s] = deg[up_col[s]];
}

// For every up-arc u -> x: its rank position r inside up(u) (number of
// members ranked below x); newcol[up_ptr[u] + r] = x, newdeg[...] = k_x,
// perm[old slot] = new slot. Quadratic in |up(u)|, which is at most sqrt(2 * edges).
__global__ void k_up_sort(const int32_t *__restrict__ src, const int2 *__restrict__ adj2,
                          const int32_t *__restrict__ upflag, const int32_t *__restrict__ upidx,
                          int64_t nnz, const int32_t *__restrict__ up_ptr,
                          const int32_t *__restrict__ up_col, const int32_t *__restrict__ upk,
                          int32_t *__restrict__ newcol, int32_t *__restrict__ newdeg,
                          int32_t *__restrict__ perm) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (!upflag[e]) continue;
    const int32_t u = src[e];
    const int2 xk = adj2[e];
    const int32_t b0 = up_ptr[u], b1 = up_ptr[u + 1];
    int32_t r = 0;
    for (int32_t j = b0; j < b1; ++j) r += rank_less(up_col[j], upk[j], xk.x, xk.y) ? 1 : 0;
    newcol[b0 + r] = xk.x;
    newdeg[b0 + r] = xk.y;
    perm[upidx[e]] = b0 + r;
  }
}

__global__ void k_tslot_remap(int32_t *__restrict__ tslot, const int32_t *__restrict__ perm,
                              int64_t nnz) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    tslot[e] = perm[tslot[e]];
}

// Segments: a down-arc w -> u (rank(u) < rank(w)) with a non-empty tail of
// up(u) above w, at a node w with up(w) non-empty (otherwise no triangle
// has w in the middle).
__global__ void k_dn_flag(const int32_t *__restrict__ src, const int32_t *__restrict__ col,
                          const int32_t *__restrict__ upflag, const int32_t *__restrict__ tslot,
                          const int32_t *__restrict__ up_ptr, int64_t nnz,
                          int32_t *__restrict__ dnflag) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t f = 0;
    if (!upflag[e]) {
      const int32_t w = src[e], u = col[e];
      const int32_t tail = up_ptr[u + 1] - tslot[e] - 1;
      f = (tail > 0 && up_ptr[w + 1] > up_ptr[w]) ? 1 : 0;
    }
    dnflag[e] = f;
  }
}

__global__ void k_dn_fill(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ src,
                          const int32_t *__restrict__ col,
                          const int32_t *__restrict__ deg, const int32_t *__restrict__ tslot,
                          const int32_t *__restrict__ up_ptr, const int32_t *__restrict__ dnflag,
                          const int32_t *__restrict__ dnidx, int32_t n, int64_t nnz,
                          int4 *__restrict__ dn, int32_t *__restrict__ dn_ptr) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int32_t ndn = nnz > 0 ? dnidx[nnz - 1] + dnflag[nnz - 1] : 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride) {
    if (dnflag[e]) {
      const int32_t u = col[e], s = tslot[e];
      dn[dnidx[e]] = make_int4(s, up_ptr[u + 1] - s - 1, deg[u] + deg[src[e]], u);
    }
  }
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += stride)
    dn_ptr[v] = (v < n && row_ptr[v] < nnz) ? dnidx[row_ptr[v]] : ndn;
}

// Upper-end slots of long-list nodes with segments: their walk adds with
// atomics, so they are cleared before each pass.
__global__ void k_zero_flag(const int32_t *__restrict__ src, const int32_t *__restrict__ upflag,
                            const int32_t *__restrict__ tslot, const int32_t *__restrict__ up_ptr,
                            const int32_t *__restrict__ dn_ptr, int64_t nnz,
                            int32_t *__restrict__ zf) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (!upflag[e]) continue;
    const int32_t a = src[e];
    const int32_t nd = dn_ptr[a + 1] - dn_ptr[a], m = up_ptr[a + 1] - up_ptr[a];
    zf[tslot[e]] = (nd > 0 && m > kTriBin2) ? 1 : 0;
  }
}

// Per arc v -> a: the triangle record that holds the credits to v, in place
// of tslot. An edge to a lower-ranked a: a's upper-end slot of {a, v},
// written by a's walk when a has segments. An edge to a higher-ranked a: the
// lower-end slot nup + slot of {v, a}, written by a's walk when {v, a} is a
// segment of a. Otherwise -1: no walk writes the record and readers skip it.
__global__ void k_trec(const int32_t *__restrict__ col, const int32_t *__restrict__ rev,
                       const int32_t *__restrict__ upflag, const int32_t *__restrict__ dn_ptr,
                       const int32_t *__restrict__ dnflag, int64_t nnz, int64_t nup,
                       int32_t *__restrict__ tslot) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = tslot[e];
    int32_t r;
    if (upflag[e]) {
      r = dnflag[rev[e]] ? (int32_t)(nup + s) : -1;
    } else {
      const int32_t a = col[e];
      r = dn_ptr[a + 1] > dn_ptr[a] ? s : -1;
    }
    tslot[e] = r;
  }
}

__global__ void k_zero_fill(const int32_t *__restrict__ zf, const int32_t *__restrict__ zidx,
                            int64_t count, int32_t *__restrict__ list) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    if (zf[i]) list[zidx[i]] = (int32_t)i;
}

// One wavefront per node: tail entries walked at w (sum of its segment lengths).
__global__ void k_dn_work(const int32_t *__restrict__ dn_ptr, const int4 *__restrict__ dn,
                          int32_t n, int64_t *__restrict__ work) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    int64_t acc = 0;
    for (int32_t i = dn_ptr[v] + lane; i < dn_ptr[v + 1]; i += 64) acc += dn[i].y;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) work[v] = acc;
  }
}

// One wavefront per node: sum of squared neighbour degrees and sum of the
// neighbours' neighbour-degree sums (with k and asum, they give N and D of
// the node in closed form).
__global__ void k_qa(const int32_t *__restrict__ row_ptr, const int2 *__restrict__ adj2,
                     const int64_t *__restrict__ asum, int32_t n, longlong2 *__restrict__ qa,
                     NbrMoments *__restrict__ nbm) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    int64_t q = 0, a2 = 0;
    double c3 = 0.0, c4 = 0.0;
    for (int32_t e = row_ptr[v] + lane; e < row_ptr[v + 1]; e += 64) {
      const int2 ad = adj2[e];
      q += (int64_t)ad.y * ad.y;
      a2 += asum[ad.x];
      const double kb = (double)ad.y, kb2 = kb * kb;
      c3 += kb2 * kb;
      c4 += kb2 * kb2;
    }
    for (int off = 32; off > 0; off >>= 1) {
      q += __shfl_xor(q, off, 64);
      a2 += __shfl_xor(a2, off, 64);
      c3 += __shfl_xor(c3, off, 64);
      c4 += __shfl_xor(c4, off, 64);
    }
    if (lane == 0) {
      qa[v] = make_longlong2(q, a2);
      nbm[v] = NbrMoments{asum[v], q, c3, c4};
    }
  }
}

// One wavefront per node: sum of neighbour degrees.
__global__ void k_asum(const int32_t *__restrict__ row_ptr, const int2 *__restrict__ adj2,
                       int32_t n, int64_t *__restrict__ asum) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    int64_t acc = 0;
    for (int32_t e = row_ptr[v] + lane; e < row_ptr[v + 1]; e += 64) acc += adj2[e].y;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) asum[v] = acc;
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 (three passes: block totals, scan of the totals in
// one workgroup, block-local scans with offsets).
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

int64_t scan_tmp_len(int64_t count) { return (count + kScanTile - 1) / kScanTile + 1; }

__device__ int32_t block_exclusive_scan(int32_t x, int32_t *sh, int32_t &total) {
  // sh: kScanThreads / 64 ints
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t incl = x;
  for (int off = 1; off < 64; off <<= 1) {
    int32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  int32_t woff = 0, tot = 0;
  for (int i = 0; i < kScanThreads / 64; ++i) {
    if (i < w) woff += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  total = tot;
  return woff + incl - x;
}

__global__ void k_scan_totals(const int32_t *__restrict__ in, int64_t count,
                              int32_t *__restrict__ totals) {
  __shared__ int32_t sh[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    if (idx < count) s += in[idx];
  }
  int32_t tot;
  block_exclusive_scan(s, sh, tot);
  if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

__global__ void k_scan_totals_single(int32_t *__restrict__ totals, int64_t nblocks) {
  __shared__ int32_t sh[kScanThreads / 64];
  int32_t carry = 0;
  for (int64_t base = 0; base < nblocks; base += kScanThreads) {
    int64_t idx = base + threadIdx.x;
    int32_t x = idx < nblocks ? totals[idx] : 0;
    int32_t tot;
    int32_t ex = block_exclusive_scan(x, sh, tot);
    if (idx < nblocks) totals[idx] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) totals[nblocks] = carry;
}

__global__ void k_scan_apply(const int32_t *__restrict__ in, int64_t count,
                             const int32_t *__restrict__ totals, int32_t *__restrict__ out) {
  __shared__ int32_t sh[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int32_t v[kScanItems];
  int32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    v[i] = idx < count ? in[idx] : 0;
    s += v[i];
  }
  int32_t tot;
  int32_t run = block_exclusive_scan(s, sh, tot) + totals[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    if (idx < count) out[idx] = run;
    run += v[i];
  }
}

hipError_t launch_exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t count,
                                     int32_t *block_tmp, int64_t block_tmp_len,
                                     hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t nb = (count + kScanTile - 1) / kScanTile;
  if (block_tmp_len < nb + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, count,
                     block_tmp);
  hipLaunchKernelGGL(k_scan_totals_single, dim3(1), dim3(kScanThreads), 0, st, block_tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, count,
                     block_tmp, out);
  return hipGetLastError();
}

static unsigned grid_for(int64_t work, int threads) {
  int64_t b = (work + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > 65535LL * 32) b = 65535LL * 32;
  return (unsigned)b;
}

// Scratch of launch_graph_prep, in ints:
//   [0, nnz)          up flags          [nnz, 2 nnz)   up indices, then cleared-slot indices
//   [2 nnz, 3 nnz)    rank keys | rank-sorted up_col, then segment indices, then cleared-slot flags
//   [3 nnz, 4 nnz)    segment flags     [4 nnz, 4 nnz + nup)   slot permutation
//   then the scan's block totals
int64_t graph_prep_tmp_len(int64_t nnz) {
  return 4 * nnz + nnz / 2 + scan_tmp_len(nnz);
}

// Everything but the zero-slot list, whose length the caller reads back
// (graph_zero_count) to size it; work[v] = tail entries walked at v.
// A simple symmetric graph has exactly nnz / 2 up-arcs; anything else is
// reported through not_symmetric before any array is filled by them.
hipError_t launch_graph_prep(Graph &g, int32_t *tmp, int64_t *work, bool &not_symmetric,
                             hipStream_t st) {
  not_symmetric = false;
  const int T = 256;
  hipLaunchKernelGGL(k_degree, dim3(grid_for(g.n, T)), dim3(T), 0, st, g.row_ptr, g.n, g.deg);
  if (g.nnz > 0) {
    const int64_t nnz = g.nnz, nup = nnz / 2;
    int32_t *upflag = tmp, *upidx = tmp + nnz, *G = tmp + 2 * nnz, *dnflag = tmp + 3 * nnz,
            *perm = tmp + 4 * nnz, *scan_tmp = tmp + 4 * nnz + nup;
    const int64_t sl = scan_tmp_len(nnz);
    hipLaunchKernelGGL(k_arc_src, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.row_ptr, g.n, nnz,
                       g.src);
    hipLaunchKernelGGL(k_arc_rev, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.row_ptr,
                       g.col_idx, g.src, g.deg, nnz, g.rev, g.adj2, upflag);
    hipError_t e = launch_exclusive_scan_i32(upflag, upidx, nnz, scan_tmp, sl, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int32_t last_idx = 0, last_flag = 0;
    if (e == hipSuccess)
      e = hipMemcpy(&last_idx, upidx + nnz - 1, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(&last_flag, upflag + nnz - 1, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    if ((int64_t)last_idx + last_flag != nup || 2 * nup != nnz) {
      not_symmetric = true;
      return hipSuccess;
    }
    hipLaunchKernelGGL(k_up_fill, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.row_ptr,
                       g.col_idx, g.rev, upflag, upidx, g.n, nnz, g.up_ptr, g.up_col,
                       g.trec);
    // rank order inside each up(u)
    int32_t *upk = G, *newcol = G + nup;
    hipLaunchKernelGGL(k_up_keys, dim3(grid_for(nup, T)), dim3(T), 0, st, g.up_col, g.deg, nup,
                       upk);
    hipLaunchKernelGGL(k_up_sort, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.src, g.adj2,
                       upflag, upidx, nnz, g.up_ptr, g.up_col, upk, newcol, g.up_deg, perm);
    e = hipMemcpyAsync(g.up_col, newcol, sizeof(int32_t) * (size_t)nup, hipMemcpyDeviceToDevice,
                       st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tslot_remap, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.trec, perm,
                       nnz);
    // segments of the triangle pass
    int32_t *dnidx = G;
    hipLaunchKernelGGL(k_dn_flag, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.src, g.col_idx,
                       upflag, g.trec, g.up_ptr, nnz, dnflag);
    e = launch_exclusive_scan_i32(dnflag, dnidx, nnz, scan_tmp, sl, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dn_fill, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.row_ptr, g.src,
                       g.col_idx, g.deg, g.trec, g.up_ptr, dnflag, dnidx, g.n, nnz, g.dn,
                       g.dn_ptr);
    hipLaunchKernelGGL(k_dn_work, dim3(grid_for((int64_t)g.n * 64, T)), dim3(T), 0, st,
                       g.dn_ptr, g.dn, g.n, work);
    // slots cleared before each pass (long lists), then their scan
    int32_t *zf = G, *zidx = upidx;
    hipLaunchKernelGGL(k_zero_flag, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.src, upflag,
                       g.trec, g.up_ptr, g.dn_ptr, nnz, zf);
    e = launch_exclusive_scan_i32(zf, zidx, nup, scan_tmp, sl, st);
    if (e != hipSuccess) return e;
    // tslot becomes the per-arc triangle record index
    hipLaunchKernelGGL(k_trec, dim3(grid_for(nnz, T)), dim3(T), 0, st, g.col_idx, g.rev, upflag,
                       g.dn_ptr, dnflag, nnz, nup, g.trec);
    hipLaunchKernelGGL(k_asum, dim3(grid_for((int64_t)g.n * 64, T)), dim3(T), 0, st,
                       g.row_ptr, g.adj2, g.n, g.asum);
    hipLaunchKernelGGL(k_qa, dim3(grid_for((int64_t)g.n * 64, T)), dim3(T), 0, st, g.row_ptr,
                       g.adj2, g.asum, g.n, g.qa, g.nbm);
  } else {
    hipLaunchKernelGGL(k_up_fill, dim3(grid_for(g.n + 1, T)), dim3(T), 0, st, g.row_ptr,
                       g.col_idx, g.rev, tmp, tmp, g.n, (int64_t)0, g.up_ptr, g.up_col,
                       g.trec);
    hipLaunchKernelGGL(k_dn_fill, dim3(grid_for(g.n + 1, T)), dim3(T), 0, st, g.row_ptr, g.src,
                       g.col_idx, g.deg, g.trec, g.up_ptr, tmp, tmp, g.n, (int64_t)0, g.dn,
                       g.dn_ptr);
    (void)hipMemsetAsync(g.asum, 0, sizeof(int64_t) * (size_t)g.n, st);
    (void)hipMemsetAsync(g.qa, 0, sizeof(longlong2) * (size_t)g.n, st);
    (void)hipMemsetAsync(g.nbm, 0, sizeof(NbrMoments) * (size_t)g.n, st);
    (void)hipMemsetAsync(work, 0, sizeof(int64_t) * (size_t)g.n, st);
  }
  return hipGetLastError();
}

// Length of the zero-slot list (after launch_graph_prep has completed).
hipError_t graph_zero_count(const Graph &g, const int32_t *tmp, int64_t &count) {
  count = 0;
  const int64_t nnz = g.nnz, nup = nnz / 2;
  if (nup <= 0) return hipSuccess;
  int32_t last_idx = 0, last_flag = 0;
  hipError_t e = hipMemcpy(&last_idx, tmp + nnz + nup - 1, sizeof(int32_t),
                           hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(&last_flag, tmp + 2 * nnz + nup - 1, sizeof(int32_t), hipMemcpyDeviceToHost);
  count = (int64_t)last_idx + last_flag;
  return e;
}

hipError_t launch_zero_list(Graph &g, const int32_t *tmp, hipStream_t st) {
  const int64_t nnz = g.nnz, nup = nnz / 2;
  if (nup <= 0 || g.n_tri_zero <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_fill, dim3(grid_for(nup, 256)), dim3(256), 0, st, tmp + 2 * nnz,
                     tmp + nnz, nup, g.tri_zero);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// degree-ordered rows of the big centres, for the super-tile pair loop: with
// the neighbours in ascending degree, the degrees inside a 64 x 64 tile are
// close, so most tiles can read their scores from a small table
// ---------------------------------------------------------------------------
__global__ void k_big_keys(const int32_t *__restrict__ row_ptr, const int2 *__restrict__ adj2,
                           const int32_t *__restrict__ big, int32_t nbig,
                           int32_t *__restrict__ kin, int32_t *__restrict__ vin,
                           int32_t *__restrict__ seg_beg, int32_t *__restrict__ seg_end) {
  for (int32_t i = blockIdx.x; i < nbig; i += gridDim.x) {
    const int32_t v = big[i], b = row_ptr[v], e = row_ptr[v + 1];
    if (threadIdx.x == 0) {
      seg_beg[i] = b;
      seg_end[i] = e;
    }
    for (int32_t x = b + threadIdx.x; x < e; x += blockDim.x) {
      kin[x] = adj2[x].y;
      vin[x] = x - b;
    }
  }
}

__global__ void k_big_pack(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ big,
                           int32_t nbig, const int32_t *__restrict__ kout,
                           const int32_t *__restrict__ vout, int2 *__restrict__ adjs) {
  for (int32_t i = blockIdx.x; i < nbig; i += gridDim.x) {
    const int32_t v = big[i], b = row_ptr[v], e = row_ptr[v + 1];
    for (int32_t x = b + threadIdx.x; x < e; x += blockDim.x) adjs[x] = make_int2(vout[x], kout[x]);
  }
}

// a big centre stores the per-arc sums of its row by sorted position: the
// reverse of the arc at sorted position x of its row finds its sum at x
__global__ void k_rrev_big(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ big,
                           int32_t nbig, const int32_t *__restrict__ rev,
                           const int2 *__restrict__ adjs, int32_t *__restrict__ rrev) {
  for (int32_t i = blockIdx.x; i < nbig; i += gridDim.x) {
    const int32_t v = big[i], b = row_ptr[v], e = row_ptr[v + 1];
    for (int32_t x = b + threadIdx.x; x < e; x += blockDim.x) rrev[rev[b + adjs[x].x]] = x;
  }
}

hipError_t launch_big_sort(Graph &g, const int32_t *big, int32_t nbig, int32_t *scratch,
                           int32_t *seg, void *temp, size_t &temp_bytes, hipStream_t st) {
  const int64_t nnz = g.nnz;
  int32_t *kin = scratch, *kout = scratch + nnz, *vin = scratch + 2 * nnz,
          *vout = scratch + 3 * nnz;
  int end_bit = 1;
  while (end_bit < 31 && (int64_t(1) << end_bit) <= (int64_t)g.info.max_degree) ++end_bit;
  if (temp == nullptr) {
    return hipcub::DeviceSegmentedRadixSort::SortPairs(
        nullptr, temp_bytes, kin, kout, vin, vout, (int)nnz, (int)nbig, seg, seg + nbig, 0,
        end_bit, st);
  }
  const unsigned grid = (unsigned)std::min<int64_t>(std::max<int32_t>(nbig, 1), 65536);
  hipLaunchKernelGGL(k_big_keys, dim3(grid), dim3(256), 0, st, g.row_ptr, g.adj2, big, nbig, kin,
                     vin, seg, seg + nbig);
  hipError_t e = hipcub::DeviceSegmentedRadixSort::SortPairs(
      temp, temp_bytes, kin, kout, vin, vout, (int)nnz, (int)nbig, seg, seg + nbig, 0, end_bit,
      st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_pack, dim3(grid), dim3(256), 0, st, g.row_ptr, big, nbig, kout, vout,
                     g.adjs);
  hipLaunchKernelGGL(k_rrev_big, dim3(grid), dim3(256), 0, st, g.row_ptr, big, nbig, g.rev,
                     g.adjs, g.rrev);
  return hipGetLastError();
}

}  // namespace efi
