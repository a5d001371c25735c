// Top-k spreaders: the k nodes of largest Expected Force ("identification of
// key nodes", the paper's title and Sec. 1). Order: EF descending, ties by
// node id ascending.
//
// EF values (and surrogate scores) are non-negative, so their IEEE bit
// patterns order like the values as unsigned integers; a value that is not
// positive (or NaN) takes key 0. Three phases, none with a device-wide sort:
//
//   1. Radix select of the k-th largest key, 8 bits at a time from the top.
//      Each pass builds one 256-bin histogram per workgroup over the keys
//      whose known high bits match (LDS atomics, no global atomics), and one
//      workgroup picks the digit where the k-th key falls. The selection
//      state lives in device memory, so the passes need no host round trip.
//   2. Order-preserving compaction of the winners: every key above the k-th
//      key's bucket, and the first `need` keys inside it in id order (ties at
//      the k-th value go to the smallest ids). Per-workgroup counts, one scan,
//      then ballot ranks keep each class in id order.
//   3. Sort of the k winners by key descending, ties by id: one workgroup
//      bitonic sort in LDS for k <= 4096; above that a stable LSD radix sort
//      (8-bit digits, ballot-ranked stable scatter), which keeps the id order
//      of equal keys that the compaction produced.
#include <mutex>

#include "ef_internal.h"

namespace efi {

namespace {

constexpr int kTkThreads = 256;     // workgroup of the streaming kernels (4 wavefronts)
constexpr int kTkSelBlocks = 1024;  // most workgroups of a selection pass
constexpr int kTkTile = 4096;       // records per workgroup in a sort pass
constexpr int kTkSmall = 4096;      // k up to this: one workgroup sorts in LDS

struct TkState {
  unsigned long long prefix;  // digits of the k-th key fixed so far
  unsigned long long mask;    // their bit positions
  long long need;             // keys still to take among those matching prefix
  int32_t done;               // exactly `need` keys match: later passes skip
  int32_t gt_total;           // keys above the bucket (set by the compaction scan)
  int32_t skip;               // sort pass: every key has the same digit
  int32_t pad[7];
};
static_assert(sizeof(TkState) == 64, "state record is one 64-byte line");

__device__ __forceinline__ unsigned long long tk_key(double v) {
  return v > 0.0 ? (unsigned long long)__double_as_longlong(v) : 0ull;
}
__device__ __forceinline__ unsigned long long tk_key(float v) {
  return v > 0.0f ? (unsigned long long)__float_as_uint(v) : 0ull;
}
template <typename V> __device__ __forceinline__ double tk_value(unsigned long long key);
template <> __device__ __forceinline__ double tk_value<double>(unsigned long long key) {
  return __longlong_as_double((long long)key);
}
template <> __device__ __forceinline__ double tk_value<float>(unsigned long long key) {
  return (double)__uint_as_float((uint32_t)key);
}

// number of set bits of m in the lanes below this one
__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__global__ void k_tk_init(TkState *st, int32_t k) {
  if (threadIdx.x == 0) {
    TkState s{};
    s.need = k;
    *st = s;
  }
}

// Phase 1: histogram of digit `shift` over the keys matching the state's prefix,
// one contiguous chunk per workgroup.
template <typename V>
__global__ __launch_bounds__(kTkThreads) void k_tk_sel_hist(const V *__restrict__ vals, int32_t n,
                                                            int32_t chunk, int shift,
                                                            const TkState *__restrict__ st,
                                                            uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[256];
  const TkState s = *st;
  if (s.done) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = min((int64_t)n, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kTkThreads) {
    const unsigned long long key = tk_key(vals[i]);
    if ((key & s.mask) == s.prefix) atomicAdd(&h[(uint32_t)(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// Phase 1: the digit of the k-th key among those matching the prefix.
__global__ __launch_bounds__(256) void k_tk_sel_pick(const uint32_t *__restrict__ hist,
                                                     int32_t nblk, int shift, TkState *st) {
  __shared__ long long c[256];
  const TkState s0 = *st;
  if (s0.done) return;
  long long sum = 0;
  for (int32_t b = 0; b < nblk; ++b) sum += hist[(size_t)b * 256 + threadIdx.x];
  c[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    TkState s = s0;
    long long need = s.need;
    int j = 255;
    for (; j > 0; --j) {
      if (c[j] >= need) break;
      need -= c[j];
    }
    s.prefix |= (unsigned long long)j << shift;
    s.mask |= 255ull << shift;
    s.need = need;
    s.done = c[j] == need ? 1 : 0;
    *st = s;
  }
}

// Phase 2: per workgroup, keys above the bucket (gt) and inside it (eq).
template <typename V>
__global__ __launch_bounds__(kTkThreads) void k_tk_count(const V *__restrict__ vals, int32_t n,
                                                         int32_t chunk,
                                                         const TkState *__restrict__ st,
                                                         int32_t *__restrict__ cnt_gt,
                                                         int32_t *__restrict__ cnt_eq) {
  __shared__ int32_t wg[4], we[4];
  const TkState s = *st;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t ng = 0, ne = 0;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = min((int64_t)n, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kTkThreads) {
    const unsigned long long m = tk_key(vals[i]) & s.mask;
    ng += m > s.prefix;
    ne += m == s.prefix;
  }
  for (int off = 32; off > 0; off >>= 1) {
    ng += __shfl_xor(ng, off, 64);
    ne += __shfl_xor(ne, off, 64);
  }
  if (lane == 0) {
    wg[w] = ng;
    we[w] = ne;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cnt_gt[blockIdx.x] = wg[0] + wg[1] + wg[2] + wg[3];
    cnt_eq[blockIdx.x] = we[0] + we[1] + we[2] + we[3];
  }
}

// Phase 2: exclusive scans of both count arrays (nblk <= 1024, one workgroup
// of 1024 threads); the gt total goes to the state.
__global__ __launch_bounds__(1024) void k_tk_count_scan(int32_t *cnt_gt, int32_t *cnt_eq,
                                                        int32_t nblk, TkState *st) {
  __shared__ int32_t a[1024], b[1024];
  const int t = threadIdx.x;
  const int32_t g0 = t < nblk ? cnt_gt[t] : 0, e0 = t < nblk ? cnt_eq[t] : 0;
  a[t] = g0;
  b[t] = e0;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t ga = t >= off ? a[t - off] : 0, eb = t >= off ? b[t - off] : 0;
    __syncthreads();
    a[t] += ga;
    b[t] += eb;
    __syncthreads();
  }
  if (t < nblk) {
    cnt_gt[t] = a[t] - g0;
    cnt_eq[t] = b[t] - e0;
  }
  if (t == 1023) st->gt_total = a[1023];
}

// Phase 2: write the winners, each class in id order: gt keys at their rank,
// eq keys after all gt keys while their rank among eq keys is below `need`.
template <typename V>
__global__ __launch_bounds__(kTkThreads) void k_tk_write(
    const V *__restrict__ vals, int32_t n, int32_t chunk, const TkState *__restrict__ st,
    const int32_t *__restrict__ off_gt, const int32_t *__restrict__ off_eq,
    unsigned long long *__restrict__ okey, int32_t *__restrict__ oid) {
  __shared__ int32_t wg[4], we[4];
  const TkState s = *st;
  const int w = threadIdx.x >> 6;
  int32_t run_g = off_gt[blockIdx.x], run_e = off_eq[blockIdx.x];
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = min((int64_t)n, lo + chunk);
  for (int64_t base = lo; base < hi; base += kTkThreads) {
    const int64_t i = base + threadIdx.x;
    unsigned long long key = 0;
    bool gt = false, eq = false;
    if (i < hi) {
      key = tk_key(vals[i]);
      const unsigned long long m = key & s.mask;
      gt = m > s.prefix;
      eq = m == s.prefix;
    }
    const unsigned long long bg = __ballot(gt), be = __ballot(eq);
    if ((threadIdx.x & 63) == 0) {
      wg[w] = __popcll(bg);
      we[w] = __popcll(be);
    }
    __syncthreads();
    int32_t pg = run_g, pe = run_e;
    for (int j = 0; j < w; ++j) {
      pg += wg[j];
      pe += we[j];
    }
    if (gt) {
      const int32_t r = pg + (int32_t)lanes_below(bg);
      okey[r] = key;
      oid[r] = (int32_t)i;
    }
    if (eq) {
      const int32_t r = pe + (int32_t)lanes_below(be);
      if (r < s.need) {
        okey[s.gt_total + r] = key;
        oid[s.gt_total + r] = (int32_t)i;
      }
    }
    run_g += wg[0] + wg[1] + wg[2] + wg[3];
    run_e += we[0] + we[1] + we[2] + we[3];
    __syncthreads();
  }
}

__device__ __forceinline__ bool tk_before(unsigned long long ka, int32_t ia, unsigned long long kb,
                                          int32_t ib) {
  return ka > kb || (ka == kb && ia < ib);
}

// Phase 3, k <= kTkSmall: bitonic sort in LDS (keys are unique with the id),
// then the outputs.
template <typename V>
__global__ __launch_bounds__(1024) void k_tk_sort_small(const unsigned long long *__restrict__ key,
                                                        const int32_t *__restrict__ id, int32_t k,
                                                        int32_t *__restrict__ nodes,
                                                        double *__restrict__ ef_out) {
  __shared__ unsigned long long sk[kTkSmall];
  __shared__ int32_t si[kTkSmall];
  int P = 2;
  while (P < k) P <<= 1;
  for (int i = threadIdx.x; i < P; i += 1024) {
    sk[i] = i < k ? key[i] : 0ull;
    si[i] = i < k ? id[i] : 0x7fffffff;  // pads sort last
  }
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < P / 2; i += 1024) {
        const int a = 2 * i - (i & (stride - 1));
        const int b = a + stride;
        const bool up = (a & size) == 0;
        const unsigned long long ka = sk[a], kb = sk[b];
        const int32_t ia = si[a], ib = si[b];
        if (up ? tk_before(kb, ib, ka, ia) : tk_before(ka, ia, kb, ib)) {
          sk[a] = kb;
          sk[b] = ka;
          si[a] = ib;
          si[b] = ia;
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += 1024) {
    nodes[i] = si[i];
    if (ef_out) ef_out[i] = tk_value<V>(sk[i]);
  }
}

// Phase 3, k > kTkSmall: one stable LSD pass on the digit 255 - byte (keys
// descending). Histogram per tile, stored digit-major for the scan.
__global__ __launch_bounds__(kTkThreads) void k_tk_rhist(const unsigned long long *__restrict__ key,
                                                         int32_t k, int shift, int32_t nblk,
                                                         uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * kTkTile;
  const int64_t hi = min((int64_t)k, lo + kTkTile);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kTkThreads)
    atomicAdd(&h[255u - ((uint32_t)(key[i] >> shift) & 255u)], 1u);
  __syncthreads();
  hist[(size_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the digit-major histogram (256 rows of nblk tiles), in
// place: four threads per digit row. A digit holding all k keys sets skip.
__global__ __launch_bounds__(1024) void k_tk_rscan(uint32_t *hist, int32_t nblk, int32_t k,
                                                   TkState *st) {
  __shared__ uint32_t part[1024];
  __shared__ uint32_t rowsum[256];
  const int t = threadIdx.x, d = t >> 2, q = t & 3;
  const int32_t per = (nblk + 3) / 4;
  const int32_t b0 = min(nblk, q * per), b1 = min(nblk, b0 + per);
  uint32_t *row = hist + (size_t)d * nblk;
  uint32_t s = 0;
  for (int32_t b = b0; b < b1; ++b) s += row[b];
  part[t] = s;
  __syncthreads();
  if (t < 256) rowsum[t] = part[4 * t] + part[4 * t + 1] + part[4 * t + 2] + part[4 * t + 3];
  __syncthreads();
  if (t == 0) {
    uint32_t acc = 0;
    int32_t same = 0;
    for (int j = 0; j < 256; ++j) {
      same |= rowsum[j] == (uint32_t)k;
      const uint32_t v = rowsum[j];
      rowsum[j] = acc;
      acc += v;
    }
    st->skip = same;
  }
  __syncthreads();
  uint32_t acc = rowsum[d];
  for (int j = 0; j < q; ++j) acc += part[4 * d + j];
  for (int32_t b = b0; b < b1; ++b) {
    const uint32_t v = row[b];
    row[b] = acc;
    acc += v;
  }
}

// Stable scatter of one tile: ranks among equal digits from wavefront
// ballots, in tile order (lanes, then wavefronts, then rounds).
__global__ __launch_bounds__(kTkThreads) void k_tk_scatter(
    const unsigned long long *__restrict__ kin, const int32_t *__restrict__ iin,
    unsigned long long *__restrict__ kout, int32_t *__restrict__ iout, int32_t k, int shift,
    const uint32_t *__restrict__ off, int32_t nblk, const TkState *__restrict__ st) {
  const int64_t lo = (int64_t)blockIdx.x * kTkTile;
  const int64_t hi = min((int64_t)k, lo + kTkTile);
  if (st->skip) {
    for (int64_t i = lo + threadIdx.x; i < hi; i += kTkThreads) {
      kout[i] = kin[i];
      iout[i] = iin[i];
    }
    return;
  }
  __shared__ uint32_t base[256];
  __shared__ uint32_t wc[4][256];
  const int t = threadIdx.x, w = t >> 6;
  base[t] = off[(size_t)t * nblk + blockIdx.x];
  wc[0][t] = wc[1][t] = wc[2][t] = wc[3][t] = 0;
  __syncthreads();
  for (int64_t b0 = lo; b0 < hi; b0 += kTkThreads) {
    const int64_t i = b0 + t;
    const bool valid = i < hi;
    unsigned long long key = 0;
    int32_t id = 0;
    uint32_t d = 0;
    if (valid) {
      key = kin[i];
      id = iin[i];
      d = 255u - ((uint32_t)(key >> shift) & 255u);
    }
    unsigned long long peers = __ballot(valid);
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long bb = __ballot(on);
      peers &= on ? bb : ~bb;
    }
    const uint32_t r = lanes_below(peers);
    if (valid && r == 0) wc[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + r;
      for (int j = 0; j < w; ++j) pos += wc[j][d];
      kout[pos] = key;
      iout[pos] = id;
    }
    __syncthreads();
    base[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
    wc[0][t] = wc[1][t] = wc[2][t] = wc[3][t] = 0;
    __syncthreads();
  }
}

template <typename V>
__global__ void k_tk_emit(const unsigned long long *__restrict__ key,
                          const int32_t *__restrict__ id, int32_t k, int32_t *__restrict__ nodes,
                          double *__restrict__ ef_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
       i += (int64_t)gridDim.x * blockDim.x) {
    nodes[i] = id[i];
    if (ef_out) ef_out[i] = tk_value<V>(key[i]);
  }
}

struct TkLayout {
  int32_t nblk = 1, chunk = 1, nsort = 0;
  size_t state = 0, hist = 0, cgt = 0, ceq = 0, k0 = 0, k1 = 0, i0 = 0, i1 = 0, rhist = 0;
  size_t bytes = 0;
};

TkLayout tk_layout(int32_t n, int32_t k) {
  TkLayout L;
  const int64_t nn = std::max<int32_t>(n, 1);
  int64_t nb = std::min<int64_t>(kTkSelBlocks, (nn + 2047) / 2048);
  int64_t chunk = (nn + nb - 1) / nb;
  chunk = (chunk + kTkThreads - 1) / kTkThreads * kTkThreads;
  L.chunk = (int32_t)chunk;
  L.nblk = (int32_t)((nn + chunk - 1) / chunk);
  L.nsort = k > kTkSmall ? (int32_t)(((int64_t)k + kTkTile - 1) / kTkTile) : 0;
  size_t p = 0;
  auto take = [&](size_t b) {
    const size_t r = p;
    p += (b + 255) & ~(size_t)255;
    return r;
  };
  const size_t kk = (size_t)std::max<int32_t>(k, 1);
  L.state = take(sizeof(TkState));
  L.hist = take(sizeof(uint32_t) * 256 * (size_t)L.nblk);
  L.cgt = take(sizeof(int32_t) * (size_t)L.nblk);
  L.ceq = take(sizeof(int32_t) * (size_t)L.nblk);
  L.k0 = take(sizeof(unsigned long long) * kk);
  L.i0 = take(sizeof(int32_t) * kk);
  if (L.nsort > 0) {
    L.k1 = take(sizeof(unsigned long long) * kk);
    L.i1 = take(sizeof(int32_t) * kk);
    L.rhist = take(sizeof(uint32_t) * 256 * (size_t)L.nsort);
  }
  L.bytes = p;
  return L;
}

template <typename V>
hipError_t topk_impl(const V *vals, int32_t n, int32_t k, void *scratch, size_t scratch_bytes,
                     int32_t *nodes, double *ef_out, hipStream_t st) {
  if (n <= 0 || k <= 0) return hipSuccess;
  if (k > n) return hipErrorInvalidValue;
  const TkLayout L = tk_layout(n, k);
  if (L.bytes > scratch_bytes) return hipErrorInvalidValue;
  char *p = (char *)scratch;
  auto *state = (TkState *)(p + L.state);
  auto *hist = (uint32_t *)(p + L.hist);
  auto *cgt = (int32_t *)(p + L.cgt);
  auto *ceq = (int32_t *)(p + L.ceq);
  auto *k0 = (unsigned long long *)(p + L.k0);
  auto *i0 = (int32_t *)(p + L.i0);
  hipLaunchKernelGGL(k_tk_init, dim3(1), dim3(64), 0, st, state, k);
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_tk_sel_hist<V>, dim3(L.nblk), dim3(kTkThreads), 0, st, vals, n, L.chunk,
                       shift, state, hist);
    hipLaunchKernelGGL(k_tk_sel_pick, dim3(1), dim3(256), 0, st, hist, L.nblk, shift, state);
  }
  hipLaunchKernelGGL(k_tk_count<V>, dim3(L.nblk), dim3(kTkThreads), 0, st, vals, n, L.chunk,
                     state, cgt, ceq);
  hipLaunchKernelGGL(k_tk_count_scan, dim3(1), dim3(1024), 0, st, cgt, ceq, L.nblk, state);
  hipLaunchKernelGGL(k_tk_write<V>, dim3(L.nblk), dim3(kTkThreads), 0, st, vals, n, L.chunk,
                     state, cgt, ceq, k0, i0);
  if (L.nsort == 0) {
    hipLaunchKernelGGL(k_tk_sort_small<V>, dim3(1), dim3(1024), 0, st, k0, i0, k, nodes, ef_out);
    return hipGetLastError();
  }
  auto *k1 = (unsigned long long *)(p + L.k1);
  auto *i1 = (int32_t *)(p + L.i1);
  auto *rh = (uint32_t *)(p + L.rhist);
  unsigned long long *ka = k0, *kb = k1;
  int32_t *ia = i0, *ib = i1;
  for (int shift = 0; shift < 64; shift += 8) {
    hipLaunchKernelGGL(k_tk_rhist, dim3(L.nsort), dim3(kTkThreads), 0, st, ka, k, shift, L.nsort,
                       rh);
    hipLaunchKernelGGL(k_tk_rscan, dim3(1), dim3(1024), 0, st, rh, L.nsort, k, state);
    hipLaunchKernelGGL(k_tk_scatter, dim3(L.nsort), dim3(kTkThreads), 0, st, ka, ia, kb, ib, k,
                       shift, rh, L.nsort, state);
    std::swap(ka, kb);
    std::swap(ia, ib);
  }
  hipLaunchKernelGGL(k_tk_emit<V>, dim3((unsigned)std::min<int64_t>((k + 255) / 256, 4096)),
                     dim3(256), 0, st, ka, ia, k, nodes, ef_out);
  return hipGetLastError();
}

}  // namespace

size_t topk_scratch_bytes(int32_t n, int32_t k) { return tk_layout(n, k).bytes; }

hipError_t launch_topk(const double *ef, int32_t n, int32_t k, void *scratch,
                       size_t scratch_bytes, int32_t *nodes, double *ef_out, hipStream_t st) {
  return topk_impl<double>(ef, n, k, scratch, scratch_bytes, nodes, ef_out, st);
}

hipError_t launch_topk_f32(const float *score, int32_t n, int32_t k, void *scratch,
                           size_t scratch_bytes, int32_t *nodes, double *score_out,
                           hipStream_t st) {
  return topk_impl<float>(score, n, k, scratch, scratch_bytes, nodes, score_out, st);
}

// ---------------------------------------------------------------------------
// Top-k for callers that cannot allocate (code under HIP graph capture,
// serving loops): the same kernels on a fixed scratch array instead of
// workspace from a graph handle. Each device holds its own copy of the array
// from module load to process end; host code reaches it only through the
// address hipGetSymbolAddress returns on that device.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)3 << 20;
constexpr int32_t kNoAllocMaxK = 65536;
constexpr int kNoAllocMaxDevices = 64;
static_assert(kNoAllocMaxK >= kTkSmall, "the no-allocation bound covers the LDS sort");

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocMaxDevices] = {};

// device address of `scratch` on the current device, resolved once per device
hipError_t noalloc_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

}  // namespace efi

extern "C" ef_status ef_topk_values_noalloc(const double *ef_in, int32_t n, int32_t k,
                                            int32_t *nodes, double *ef, uint32_t flags,
                                            void *hip_stream) {
  using namespace efi;
  if (n < 0 || k < 0 || k > n) {
    set_error("ef_topk_values_noalloc: need 0 <= k <= n (k=%d, n=%d)", k, n);
    return EF_ERR_ARG;
  }
  if (k > kNoAllocMaxK) {
    set_error("ef_topk_values_noalloc: k=%d above the fixed-scratch limit %d", k, kNoAllocMaxK);
    return EF_ERR_ARG;
  }
  if (flags != EF_OUT_DEVICE) {
    set_error("ef_topk_values_noalloc: flags must be EF_OUT_DEVICE (device outputs), got 0x%x",
              flags);
    return EF_ERR_ARG;
  }
  if (k == 0) return EF_OK;
  if (!ef_in || !nodes) {
    set_error("ef_topk_values_noalloc: null values or output");
    return EF_ERR_ARG;
  }
  const size_t need = topk_scratch_bytes(n, k);
  if (need > kNoAllocScratchBytes) {
    set_error("ef_topk_values_noalloc: n=%d, k=%d need %zu scratch bytes, above %zu", n, k, need,
              kNoAllocScratchBytes);
    return EF_ERR_ARG;
  }
  void *ptr = nullptr;
  hipError_t e = noalloc_scratch(&ptr);
  if (e != hipSuccess) return hip_status(e, "fixed scratch address");
  e = launch_topk(ef_in, n, k, ptr, kNoAllocScratchBytes, nodes, ef, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_status(e, "top-k");
  return EF_OK;
}
