// Graph preprocessing on the device: degrees, arc sources, reverse arcs, the
// packed (id, degree) adjacency, neighbour-degree sums and the
// degree-oriented half adjacency used by the triangle pass.
//
// The orientation ranks nodes by (degree, id): rank(a) < rank(b) when
// k_a < k_b, or k_a == k_b and a < b. up(u) = {w in N(u) : rank(w) > rank(u)}
// keeps every undirected edge exactly once and bounds |up(u)| by
// sqrt(2 * edges), which keeps the triangle pass short on skewed graphs.
#include "ef_internal.h"

namespace efi {

__device__ __forceinline__ bool rank_less(int32_t a, int32_t ka, int32_t b, int32_t kb) {
  return ka < kb || (ka == kb && a < b);
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

// flags_scan_tmp: 2 * nnz + scan_tmp_len(nnz) ints of scratch.
hipError_t launch_graph_prep(Graph &g, int32_t *tmp, hipStream_t st) {
  const int T = 256;
  hipLaunchKernelGGL(k_degree, dim3(grid_for(g.n, T)), dim3(T), 0, st, g.row_ptr, g.n, g.deg);
  if (g.nnz > 0) {
    int32_t *upflag = tmp, *upidx = tmp + g.nnz, *scan_tmp = tmp + 2 * g.nnz;
    hipLaunchKernelGGL(k_arc_src, dim3(grid_for(g.nnz, T)), dim3(T), 0, st, g.row_ptr, g.n,
                       g.nnz, g.src);
    hipLaunchKernelGGL(k_arc_rev, dim3(grid_for(g.nnz, T)), dim3(T), 0, st, g.row_ptr,
                       g.col_idx, g.src, g.deg, g.nnz, g.rev, g.adj2, upflag);
    hipError_t e = launch_exclusive_scan_i32(upflag, upidx, g.nnz, scan_tmp,
                                             scan_tmp_len(g.nnz), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_up_fill, dim3(grid_for(g.nnz, T)), dim3(T), 0, st, g.row_ptr,
                       g.col_idx, g.rev, upflag, upidx, g.n, g.nnz, g.up_ptr, g.up_col,
                       g.tslot);
    hipLaunchKernelGGL(k_asum, dim3(grid_for((int64_t)g.n * 64, T)), dim3(T), 0, st,
                       g.row_ptr, g.adj2, g.n, g.asum);
  } else {
    hipLaunchKernelGGL(k_up_fill, dim3(grid_for(g.n + 1, T)), dim3(T), 0, st, g.row_ptr,
                       g.col_idx, g.rev, tmp, tmp, g.n, (int64_t)0, g.up_ptr, g.up_col,
                       g.tslot);
    (void)hipMemsetAsync(g.asum, 0, sizeof(int64_t) * (size_t)g.n, st);
  }
  return hipGetLastError();
}

}  // namespace efi
