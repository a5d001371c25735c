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
//
// Listing: nodes are ranked by (degree, id); a triangle u < w < x (by rank) is
// found once, at u, as x in up(u) and up(w), where up(.) is the rank-oriented
// out-list. up(u) is hashed in LDS (id -> degree, position) and the lists
// up(w), w in up(u), are walked as one concatenated sequence ("segments"),
// 64 consecutive entries per wavefront step. Short up(u): one wavefront per u.
// Longer up(u): one workgroup per u, each wavefront walking a contiguous
// share of the sequence. Credits:
//   u  - lane registers (floating point), reduced at the end  -> Z[u], ZT[u]
//   w  - LDS add at w's position in up(u)
//   x  - LDS add at x's position in up(u)
// The LDS credit slots are integers (see Credit), so concurrent adds are exact
// and order-independent: results are bitwise reproducible. The slots are
// written to Y[slot], YT[slot] for the up-arc slots of u.
#include "common.cuh"

namespace efi {

constexpr double kFix = 1099511627776.0;  // 2^40
constexpr int kPosBits = 12;              // position in up(u) < 4096
static_assert(kTriBin2 <= (1 << kPosBits), "position field too narrow");
static_assert(kMaxDegree < (1u << (32 - kPosBits)), "degree field too narrow");

__device__ __forceinline__ int32_t pack_kp(int32_t k, int32_t pos) {
  return (int32_t)(((uint32_t)k << kPosBits) | (uint32_t)pos);
}
__device__ __forceinline__ int32_t unpack_k(int32_t v) { return (int32_t)((uint32_t)v >> kPosBits); }

template <typename T> __device__ __forceinline__ long long to_fix(T v) {
  return __double2ll_rn((double)v * kFix);
}

// Integer credit slots, 2^-40 units on output.
// FP32: delta < 0 is a float with 2 <= |delta| < 2^7 (log2 units, degrees
//   below kMaxDegree), so its ulp is >= 2^-22 and |delta| * 2^24 is an exact
//   integer below 2^31. A slot holds one word, count << 44 plus the sum of
//   those integers; at most kTriBin2 = 2^11 credits land in a slot, so the
//   sum stays below 2^42 and one 64-bit add records credit and count.
// FP64: the credit rounded to 2^-40 in one 64-bit slot, the count in a
//   separate 32-bit slot.
template <typename T> struct Credit;
template <> struct Credit<float> {
  static constexpr bool kPacked = true;
  __device__ static void add(unsigned long long *acc, int32_t *, int32_t slot, float dl) {
    atomicAdd(&acc[slot], (1ull << 44) + (unsigned long long)(uint32_t)(-dl * 16777216.0f));
  }
  __device__ static void load(const unsigned long long *acc, const int32_t *, int32_t slot,
                              long long &y, int32_t &yt) {
    const unsigned long long w = acc[slot];
    y = -(long long)((w & ((1ull << 44) - 1)) << 16);
    yt = (int32_t)(w >> 44);
  }
};
template <> struct Credit<double> {
  static constexpr bool kPacked = false;
  __device__ static void add(unsigned long long *acc, int32_t *cnt, int32_t slot, double dl) {
    atomicAdd(&acc[slot], (unsigned long long)to_fix(dl));
    atomicAdd(&cnt[slot], 1);
  }
  __device__ static void load(const unsigned long long *acc, const int32_t *cnt, int32_t slot,
                              long long &y, int32_t &yt) {
    y = (long long)acc[slot];
    yt = cnt[slot];
  }
};

// Count-only pass (triangle counts per node and up-arc, no score terms): a
// tag type whose sums, deltas and credits reduce to counting.
struct TriCount {};
struct NoSum {};
__device__ __forceinline__ NoSum wave_sum(NoSum x) { return x; }
__device__ __forceinline__ void acc_merge(NoSum &, NoSum) {}
template <> struct SumT<TriCount> {
  using type = NoSum;
  __device__ static void add_term(NoSum &, TriCount) {}
  __device__ static void store(const NoSum &, void *, int64_t) {}
};
template <> __device__ __forceinline__ TriCount tri_delta<TriCount>(int32_t) { return TriCount{}; }
__device__ __forceinline__ long long to_fix(TriCount) { return 0; }
template <> struct Credit<TriCount> {
  static constexpr bool kPacked = true;
  __device__ static void add(unsigned long long *acc, int32_t *, int32_t slot, TriCount) {
    atomicAdd(&acc[slot], 1ull << 44);
  }
  __device__ static void load(const unsigned long long *acc, const int32_t *, int32_t slot,
                              long long &y, int32_t &yt) {
    y = 0;
    yt = (int32_t)(acc[slot] >> 44);
  }
};

// LDS state of one u:
//   hkey[SLOTS]   ids x of up(u) (LdsHash), hval[slot] = k_x << kPosBits |
//                 position of x in up(u)
//   seg[MAXM]     per non-empty up(w): {first index of up(w) in up_col minus
//                 its first index in the concatenated sequence,
//                 k_w << kPosBits | position of w in up(u)}
//   segp[MAXM+1]  first concatenated index of each segment; segp[nseg] = total
//   acc, cnt      credit slots by position in up(u)
//   flg[kFlg]     per wavefront: segment-start flags of the current step
template <typename T, int SLOTS, int MAXM> struct TriLds {
  static_assert(SLOTS >= 2 * MAXM, "the hash set of up(u) must stay at most half full");
  __align__(16) int32_t hkey[SLOTS];
  int32_t hval[SLOTS];
  int2 seg[MAXM];
  int32_t segp[MAXM + 1];
  unsigned long long acc[MAXM];
  int32_t cnt[Credit<T>::kPacked ? 1 : MAXM];
};

// Build the hash of up(u) and the segment table with NT threads (one
// wavefront, or the workgroup); `part` holds 2 * NT/64 ints of scratch.
// Returns the segment count and the sequence length.
template <int SLOTS, int NT>
__device__ __forceinline__ void tri_setup(const int32_t *__restrict__ up_ptr,
                                          const int32_t *__restrict__ up_col,
                                          const int32_t *__restrict__ deg, int32_t u0, int32_t m,
                                          int tid, int32_t *hkey, int32_t *hval, int2 *seg,
                                          int32_t *segp,
                                          int32_t *part, int32_t &nseg_out, int32_t &total_out,
                                          int32_t &myslot) {
  constexpr int NW = NT / 64;
  const int lane = tid & 63, wv = tid >> 6;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int32_t nseg = 0, run = 0;
  for (int c = 0; c < m; c += NT) {
    const int i = c + tid;
    int32_t x = 0, w0 = 0, len = 0, kx = 0;
    if (i < m) {
      x = up_col[u0 + i];
      w0 = up_ptr[x];
      len = up_ptr[x + 1] - w0;
      kx = deg[x];
      myslot = LdsHash<SLOTS>::insert(hkey, x);
      hval[myslot] = pack_kp(kx, i);
    }
    const unsigned long long nz = __ballot(len > 0);
    int32_t incl = len;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    int32_t pre_n = 0, pre_l = 0, tot_n, tot_l;
    if constexpr (NW == 1) {
      tot_n = __popcll(nz);
      tot_l = __shfl(incl, 63, 64);
    } else {
      if (lane == 63) {
        part[2 * wv] = __popcll(nz);
        part[2 * wv + 1] = incl;
      }
      __syncthreads();
      tot_n = 0;
      tot_l = 0;
      for (int w = 0; w < NW; ++w) {
        const int32_t a = part[2 * w], b = part[2 * w + 1];
        if (w < wv) {
          pre_n += a;
          pre_l += b;
        }
        tot_n += a;
        tot_l += b;
      }
    }
    if (len > 0) {
      const int32_t slot = nseg + pre_n + __popcll(nz & lt_mask);
      const int32_t start = run + pre_l + incl - len;
      seg[slot] = make_int2(w0 - start, pack_kp(kx, i));
      segp[slot] = start;
    }
    nseg += tot_n;
    run += tot_l;
    if constexpr (NW > 1) __syncthreads();
  }
  if (tid == 0) segp[nseg] = run;
  nseg_out = nseg;
  total_out = run;
}

// One wavefront walks entries [beg, end) of u's concatenated up(w) lists,
// 64 consecutive entries per step (segment of each lane: seg_walk). A hit
// (x in up(u)) is appended to the wavefront's LDS queue as two words,
// {sigma, pos(w) | pos(x) << 16}; whenever 64 hits are queued they are
// scored and credited with every lane busy, so the hit path does not run
// divergently on almost every step (about 6% of the entries are hits).
constexpr int kQueue = 128;

template <typename T, int SLOTS, int MAXM>
__device__ __forceinline__ void tri_walk(const int32_t *__restrict__ up_col,
                                         TriLds<T, SLOTS, MAXM> &L, int32_t *flg, int2 *hq,
                                         int32_t nseg, int32_t beg, int32_t end, int32_t ku,
                                         typename SumT<T>::type &accu, int64_t &cntu) {
  using S = SumT<T>;
  constexpr int32_t kPosMask = (1 << kPosBits) - 1;
  const int lane = threadIdx.x & 63;
  const int2 *seg = L.seg;
  const int32_t *hkey = L.hkey;
  const int32_t *hval = L.hval;
  int32_t qn = 0;  // queued hits (uniform)
  // score and credit hq[qn - cnt .. qn) on lanes 0 .. cnt-1
  auto drain = [&](int32_t cnt) {
    wave_sync();
    if (lane < cnt) {
      const int2 h = hq[qn - cnt + lane];
      const T dl = tri_delta<T>(h.x);
      S::add_term(accu, dl);
      ++cntu;
      Credit<T>::add(L.acc, L.cnt, h.y >> 16, dl);
      Credit<T>::add(L.acc, L.cnt, h.y & 0xFFFF, dl);
    }
    qn -= cnt;
    wave_sync();
  };
  seg_walk<4>(
      L.segp, nseg, beg, end, flg,
      [&](int32_t sg, int32_t idx) {
        const int2 sv = seg[sg];
        return make_int2(up_col[sv.x + idx], sv.y);
      },
      [&](int32_t, int32_t, int2 xv, bool ok) {
        const int32_t slot = ok ? LdsHash<SLOTS>::find(hkey, xv.x) : -1;
        const bool hit = slot >= 0;
        const unsigned long long m = __ballot(hit);
        if (hit) {
          const int32_t ev = hval[slot];
          const int32_t rank = (int32_t)__builtin_amdgcn_mbcnt_hi(
              (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          hq[qn + rank] = make_int2(ku + unpack_k(xv.y) + unpack_k(ev),
                                    (xv.y & kPosMask) | ((ev & kPosMask) << 16));
        }
        qn += __popcll(m);
        if (qn >= 64) drain(64);
      });
  if (qn > 0) drain(qn);
}

template <typename T, int SLOTS, int MAXM>
__device__ __forceinline__ void tri_clear_acc(TriLds<T, SLOTS, MAXM> &L, int32_t m, int tid,
                                              int nt) {
  for (int i = tid; i < m; i += nt) {
    L.acc[i] = 0ull;
    if constexpr (!Credit<T>::kPacked) L.cnt[i] = 0;
  }
}

template <typename T, int SLOTS, int MAXM>
__device__ __forceinline__ void tri_clear(TriLds<T, SLOTS, MAXM> &L, int32_t m, int tid, int nt) {
  for (int i = tid; i < SLOTS; i += nt) L.hkey[i] = -1;
  for (int i = tid; i < m; i += nt) {
    L.acc[i] = 0ull;
    if constexpr (!Credit<T>::kPacked) L.cnt[i] = 0;
  }
}

template <typename T, int SLOTS, int MAXM>
__device__ __forceinline__ void tri_store(const TriLds<T, SLOTS, MAXM> &L, int32_t u0, int32_t m,
                                          int tid, int nt, long long *Y, int32_t *YT) {
  for (int i = tid; i < m; i += nt) {
    long long y;
    int32_t yt;
    Credit<T>::load(L.acc, L.cnt, i, y, yt);
    Y[u0 + i] = y;
    YT[u0 + i] = yt;
  }
}

// One node u per wavefront (short up(u)); WPB wavefronts per workgroup, each
// with its own LDS state.
template <typename T, int SLOTS, int MAXM, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_tri_wave(
    const int32_t *__restrict__ up_ptr, const int32_t *__restrict__ up_col,
    const int32_t *__restrict__ deg, const int32_t *__restrict__ nodes, int64_t count,
    long long *__restrict__ Y, int32_t *__restrict__ YT, void *__restrict__ Z,
    int64_t *__restrict__ ZT) {
  using S = SumT<T>;
  using Acc = typename S::type;
  __shared__ TriLds<T, SLOTS, MAXM> lds[WPB];
  __shared__ int32_t flg_s[WPB][kFlg];
  __shared__ int2 hq_s[WPB][kQueue];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  TriLds<T, SLOTS, MAXM> &L = lds[wv];
  int32_t *flg = flg_s[wv];
  flg[lane] = 0;
  const int64_t nwaves = (int64_t)gridDim.x * WPB;
  // the hash is cleared once; afterwards each lane empties the one slot it
  // filled (|up(u)| <= 64), so a short list does not pay for the whole table
  static_assert(MAXM <= 64, "one up(u) entry per lane");
  for (int i = lane; i < SLOTS; i += 64) L.hkey[i] = -1;
  for (int64_t it = (int64_t)blockIdx.x * WPB + wv; it < count; it += nwaves) {
    const int32_t u = nodes[it];
    const int32_t u0 = up_ptr[u], m = up_ptr[u + 1] - u0, ku = deg[u];
    tri_clear_acc(L, m, lane, 64);
    wave_sync();
    int32_t nseg, total, myslot = -1;
    tri_setup<SLOTS, 64>(up_ptr, up_col, deg, u0, m, lane, L.hkey, L.hval, L.seg, L.segp, nullptr,
                         nseg, total, myslot);
    wave_sync();
    Acc accu = Acc();
    int64_t cntu = 0;
    tri_walk<T, SLOTS, MAXM>(up_col, L, flg, hq_s[wv], nseg, 0, total, ku, accu, cntu);
    accu = wave_sum(accu);
    cntu = wave_sum_i64(cntu);
    if (lane == 0) {
      S::store(accu, Z, u);
      ZT[u] = cntu;
    }
    tri_store(L, u0, m, lane, 64, Y, YT);
    if (myslot >= 0) L.hkey[myslot] = -1;
    wave_sync();
  }
}

// One node u per workgroup of WPB wavefronts sharing one LDS state; each
// wavefront walks a contiguous share of the sequence.
template <typename T, int SLOTS, int MAXM, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_tri_block(
    const int32_t *__restrict__ up_ptr, const int32_t *__restrict__ up_col,
    const int32_t *__restrict__ deg, const int32_t *__restrict__ nodes, int64_t count,
    long long *__restrict__ Y, int32_t *__restrict__ YT, void *__restrict__ Z,
    int64_t *__restrict__ ZT) {
  using S = SumT<T>;
  using Acc = typename S::type;
  constexpr int NT = 64 * WPB;
  __shared__ TriLds<T, SLOTS, MAXM> L;
  __shared__ int32_t flg_s[WPB][kFlg];
  __shared__ int2 hq_s[WPB][kQueue];
  __shared__ int32_t part[2 * WPB];
  __shared__ Acc sh_acc[WPB];
  __shared__ int64_t sh_cnt[WPB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int32_t *flg = flg_s[wv];
  flg[lane] = 0;
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t u = nodes[it];
    const int32_t u0 = up_ptr[u], m = up_ptr[u + 1] - u0, ku = deg[u];
    tri_clear(L, m, tid, NT);
    __syncthreads();
    int32_t nseg, total;
    int32_t myslot;
    tri_setup<SLOTS, NT>(up_ptr, up_col, deg, u0, m, tid, L.hkey, L.hval, L.seg, L.segp, part, nseg,
                         total, myslot);
    __syncthreads();
    // contiguous shares, multiples of 64 entries
    const int32_t steps = (total + 63) >> 6;
    const int32_t beg = (int32_t)(((int64_t)steps * wv / WPB) << 6);
    const int32_t fin = (int32_t)(((int64_t)steps * (wv + 1) / WPB) << 6);
    Acc accu = Acc();
    int64_t cntu = 0;
    tri_walk<T, SLOTS, MAXM>(up_col, L, flg, hq_s[wv], nseg, beg, fin < total ? fin : total, ku,
                             accu, cntu);
    accu = wave_sum(accu);
    cntu = wave_sum_i64(cntu);
    if (lane == 0) {
      sh_acc[wv] = accu;
      sh_cnt[wv] = cntu;
    }
    __syncthreads();
    if (tid == 0) {
      Acc a = sh_acc[0];
      int64_t cs = sh_cnt[0];
      for (int w = 1; w < WPB; ++w) {
        acc_merge(a, sh_acc[w]);
        cs += sh_cnt[w];
      }
      S::store(a, Z, u);
      ZT[u] = cs;
    }
    tri_store(L, u0, m, tid, NT, Y, YT);
    __syncthreads();
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
    hipLaunchKernelGGL((k_tri_wave<T, 256, 64, 4>), dim3(cap_blocks((counts[0] + 3) / 4, 1 << 20)),
                       dim3(256), 0, st, g.up_ptr, g.up_col, g.deg, lists[0], counts[0], Y, YT,
                       Z, ZT);
  if (counts[1] > 0)
    hipLaunchKernelGGL((k_tri_block<T, 2048, 512, 8>), dim3(cap_blocks(counts[1], 1 << 20)),
                       dim3(512), 0, st, g.up_ptr, g.up_col, g.deg, lists[1], counts[1], Y, YT,
                       Z, ZT);
  if (counts[2] > 0)
    hipLaunchKernelGGL((k_tri_block<T, 8192, 2048, 16>), dim3(cap_blocks(counts[2], 1 << 20)),
                       dim3(1024), 0, st, g.up_ptr, g.up_col, g.deg, lists[2], counts[2], Y, YT,
                       Z, ZT);
  if (counts[3] > 0)
    hipLaunchKernelGGL(k_tri_long<T>, dim3(cap_blocks(counts[3], 1 << 20)), dim3(64), 0, st,
                       g.up_ptr, g.up_col, g.deg, lists[3], counts[3], Y, YT, Z, ZT);
  return hipGetLastError();
}

hipError_t launch_triangles_count(const Graph &g, long long *Y, int32_t *YT, int64_t *ZT,
                                  hipStream_t st) {
  const int32_t *lists[4] = {g.tri_list[0], g.tri_list[1], g.tri_list[2], g.tri_list[3]};
  return tri_impl<TriCount>(g, lists, g.n_tri, Y, YT, nullptr, ZT, st);
}

hipError_t launch_triangles(const Graph &g, ef_prec prec, long long *Y, int32_t *YT, void *Z,
                            int64_t *ZT, hipStream_t st) {
  const int32_t *lists[4] = {g.tri_list[0], g.tri_list[1], g.tri_list[2], g.tri_list[3]};
  if (prec == EF_PREC_FP64) return tri_impl<double>(g, lists, g.n_tri, Y, YT, Z, ZT, st);
  return tri_impl<float>(g, lists, g.n_tri, Y, YT, Z, ZT, st);
}

}  // namespace efi
