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
// Listing: nodes are ranked by (degree, id) and every up(.) list (members of
// higher rank) is stored in rank order. A triangle u < w < x (by rank) is
// found once, at its middle node w: x lies in up(w) and in the tail of up(u)
// above w. up(w) is hashed in LDS (id -> degree, position), and the tails of
// up(u) for the lower neighbours u of w ("segments", built with the graph)
// are walked as one concatenated sequence, 64 consecutive entries per
// wavefront step. Each membership test is one pair (w, x) inside some up(u),
// so the pass makes sum_u C(|up(u)|, 2) tests, against
// sum_w |up(w)| * |down(w)| for a listing at the lowest node.
// Credits, per triangle:
//   w  - lane registers (floating point), reduced at the end  -> Z[w], ZT[w]
//   x  - LDS add at x's position in up(w)  -> upper-end record Y[slot of {w, x}]
//   u  - LDS add at the segment's index    -> lower-end record Y[nup + slot of {u, w}]
// The LDS credit slots are integers (see Credit), so concurrent adds are exact
// and order-independent: results are bitwise reproducible. Segments are taken
// in chunks of at most MAXS; the credits to x are added to their slots after
// every chunk, which bounds the credits an LDS slot holds by 2^11.
#include "common.cuh"

namespace efi {

constexpr int kPosBits = 12;              // position in up(u) < 4096
static_assert(kTriBin2 <= (1 << kPosBits), "position field too narrow");
static_assert(kMaxDegree < (1u << (32 - kPosBits)), "degree field too narrow");

__device__ __forceinline__ int32_t pack_kp(int32_t k, int32_t pos) {
  return (int32_t)(((uint32_t)k << kPosBits) | (uint32_t)pos);
}
__device__ __forceinline__ int32_t unpack_k(int32_t v) { return (int32_t)((uint32_t)v >> kPosBits); }

template <typename T> __device__ __forceinline__ long long to_fix(T v) {
  return __double2ll_rn((double)v * kTriFix);
}

// Integer credit slots in LDS, 2^-36 units on output (TriSlot).
// FP32: delta < 0 is a float with 2 <= |delta| < 2^7 (log2 units, degrees
//   below kMaxDegree), so its ulp is >= 2^-22 and |delta| * 2^24 is an exact
//   integer below 2^31. A slot holds one word, count << 44 plus the sum of
//   those integers; at most 2^11 credits land in a slot before it is flushed
//   (a segment's hits are members of up(w), |up(w)| <= kTriBin2 = 2^11; x
//   gets at most one credit per segment of a chunk, MAXS <= 2^11), so the
//   sum stays below 2^42 and one 64-bit add records credit and count.
// FP64: the credit rounded to 2^-36 in one 64-bit slot, the count in a
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
    y = -(long long)((w & ((1ull << 44) - 1)) << 12);
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

// LDS state of one w:
//   hkey[SLOTS]   ids x of up(w) (LdsHash), hval[slot] = k_x << kPosBits |
//                 position of x in up(w)
//   seg[MAXS]     per segment of the chunk: {first index of the tail in up_col
//                 minus its first index in the concatenated sequence, k_u + k_w}
//   segp[MAXS+1]  first concatenated index of each segment; segp[nseg] = total
//   sslot[MAXS]   slot of {u, w} in up(u): the segment's lower-end slot
//   acc, cnt      credits to x by position in up(w)
//   sacc, scnt    credits to u by segment
template <typename T, int SLOTS, int MAXM, int MAXS> struct TriLds {
  static_assert(SLOTS >= 2 * MAXM, "the hash set of up(w) must stay at most half full");
  static_assert(MAXM <= (1 << 11) && MAXS <= (1 << 11), "credit slots hold at most 2^11 credits");
  __align__(16) int32_t hkey[SLOTS];
  int32_t hval[SLOTS];
  int2 seg[MAXS];
  int32_t segp[MAXS + 1];
  int32_t sslot[MAXS];
  unsigned long long acc[MAXM];
  unsigned long long sacc[MAXS];
  int32_t cnt[Credit<T>::kPacked ? 1 : MAXM];
  int32_t scnt[Credit<T>::kPacked ? 1 : MAXS];
};

// Hash up(w) (m entries from w0) with NT threads; returns the slot this
// thread filled last (-1 if none).
template <int SLOTS, int NT>
__device__ __forceinline__ int32_t tri_hash(const int32_t *__restrict__ up_col,
                                            const int32_t *__restrict__ up_deg, int32_t w0,
                                            int32_t m, int tid, int32_t *hkey, int32_t *hval) {
  int32_t myslot = -1;
  for (int32_t i = tid; i < m; i += NT) {
    const int32_t x = up_col[w0 + i];
    myslot = LdsHash<SLOTS>::insert(hkey, x);
    hval[myslot] = pack_kp(up_deg[w0 + i], i);
  }
  return myslot;
}

// Segment table of one chunk: entry e (a dn record, meaningful for
// tid < cnt <= NT; every segment is non-empty). Returns the concatenated
// length (workgroup form: every thread calls it; `part` holds NT/64 ints).
template <int NT, typename L>
__device__ __forceinline__ int32_t tri_segs(int4 e, int32_t cnt, int tid, L &lds, int32_t *part) {
  int32_t total;
  const int32_t start = group_excl_scan<NT>(tid < cnt ? e.y : 0, part, total);
  if (tid < cnt) {
    lds.seg[tid] = make_int2(e.x + 1 - start, e.z);
    lds.segp[tid] = start;
    lds.sslot[tid] = e.x;
  }
  if (tid == 0) lds.segp[cnt] = total;
  return total;
}

// One wavefront walks entries [beg, end) of the chunk's concatenated tails,
// 64 consecutive entries per step (segment of each lane: seg_walk). A hit
// (x in up(w)) is appended to the wavefront's LDS queue as two words,
// {sigma, segment | pos(x) << 16}; whenever 64 hits are queued they are
// scored and credited with every lane busy, so the hit path does not run
// divergently on almost every step.
constexpr int kQueue = 128;
// tri_walk drains once the queue holds 64 hits, so up to 63 wait while a
// wavefront appends up to 64 more: indices reach 126
static_assert(kQueue >= 127, "the hit queue must hold 63 waiting + 64 new hits");

template <typename T, int SLOTS, int MAXM, int MAXS>
__device__ __forceinline__ void tri_walk(const int32_t *__restrict__ up_col,
                                         TriLds<T, SLOTS, MAXM, MAXS> &L, int32_t *flg, int2 *hq,
                                         int32_t nseg, int32_t beg, int32_t end,
                                         typename SumT<T>::type &accw, int64_t &cntw) {
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
      S::add_term(accw, dl);
      ++cntw;
      Credit<T>::add(L.acc, L.cnt, h.y >> 16, dl);
      Credit<T>::add(L.sacc, L.scnt, h.y & 0xFFFF, dl);
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
      [&](int32_t sg, int32_t, int2 xv, bool ok) {
        const int32_t slot = ok ? LdsHash<SLOTS>::find(hkey, xv.x) : -1;
        const bool hit = slot >= 0;
        const unsigned long long m = __ballot(hit);
        if (hit) {
          const int32_t ev = hval[slot];
          const int32_t rank = (int32_t)__builtin_amdgcn_mbcnt_hi(
              (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          hq[qn + rank] = make_int2(xv.y + unpack_k(ev), sg | ((ev & kPosMask) << 16));
        }
        qn += __popcll(m);
        if (qn >= 64) drain(64);
      });
  if (qn > 0) drain(qn);
}

// After a chunk: the credits to u go to the segments' lower-end slots, the
// credits to x are stored (first chunk) or added to w's upper-end slots.
// Clears both for the next chunk.
template <typename T, int SLOTS, int MAXM, int MAXS>
__device__ __forceinline__ void tri_flush(TriLds<T, SLOTS, MAXM, MAXS> &L, int32_t cnt, int32_t w0,
                                          int32_t m, bool first, int tid, int nt, int64_t nup,
                                          TriSlot *Y) {
  for (int32_t i = tid; i < cnt; i += nt) {
    TriSlot r{0, 0, 0};
    Credit<T>::load(L.sacc, L.scnt, i, r.y, r.t);
    Y[nup + L.sslot[i]] = r;
    L.sacc[i] = 0ull;
    if constexpr (!Credit<T>::kPacked) L.scnt[i] = 0;
  }
  for (int32_t i = tid; i < m; i += nt) {
    TriSlot r{0, 0, 0};
    Credit<T>::load(L.acc, L.cnt, i, r.y, r.t);
    if (!first) {
      const TriSlot o = Y[w0 + i];
      r.y += o.y;
      r.t += o.t;
    }
    Y[w0 + i] = r;
    L.acc[i] = 0ull;
    if constexpr (!Credit<T>::kPacked) L.cnt[i] = 0;
  }
}

template <typename T, int SLOTS, int MAXM, int MAXS>
__device__ __forceinline__ void tri_clear_credits(TriLds<T, SLOTS, MAXM, MAXS> &L, int tid,
                                                  int nt) {
  for (int i = tid; i < MAXM; i += nt) {
    L.acc[i] = 0ull;
    if constexpr (!Credit<T>::kPacked) L.cnt[i] = 0;
  }
  for (int i = tid; i < MAXS; i += nt) {
    L.sacc[i] = 0ull;
    if constexpr (!Credit<T>::kPacked) L.scnt[i] = 0;
  }
}

struct TriArgs {
  const int32_t *up_ptr, *up_col, *up_deg, *dn_ptr;
  const int4 *dn;
  int64_t nup;
  TriSlot *Y;
  void *Z;
  int64_t *ZT;
};

// One node w per wavefront (|up(w)| <= 64, short walk), chunks of 64
// segments, with the wavefront's own LDS state. rc = {w, first up slot, first
// segment, |up(w)| | segments << 16}. On entry the hash holds no key, flg is
// zero and the credit slots are clear (tri_wave_init); on return too: each
// lane empties the one hash slot it filled, so a short list does not pay for
// the whole table.
template <typename T, int SLOTS, int MAXM>
__device__ __forceinline__ void tri_wave_node(const TriArgs &A, const int4 rc,
                                              TriLds<T, SLOTS, MAXM, 64> &L, int32_t *flg,
                                              int2 *hq) {
  using S = SumT<T>;
  using Acc = typename S::type;
  constexpr int MAXS = 64;
  static_assert(MAXM <= 64, "one up(w) entry per lane");
  const int lane = threadIdx.x & 63;
  const int32_t w = rc.x, w0 = rc.y, d0 = rc.z, m = rc.w & 0xFFFF, nd = rc.w >> 16;
  // m >= 1 and nd >= 1 for every listed node: clamped indices stay in
  // w's rows, and every lane loads without a branch
  const int32_t ui = w0 + (lane < m ? lane : m - 1);
  const int32_t x = A.up_col[ui], kx = A.up_deg[ui];
  int4 sg = A.dn[d0 + (lane < nd ? lane : nd - 1)];
  wave_sync();
  int32_t myslot = -1;
  if (lane < m) {
    myslot = LdsHash<SLOTS>::insert(L.hkey, x);
    L.hval[myslot] = pack_kp(kx, lane);
  }
  Acc accw = Acc();
  int64_t cntw = 0;
  for (int32_t c0 = 0; c0 < nd; c0 += MAXS) {
    const int32_t cnt = nd - c0 < MAXS ? nd - c0 : MAXS;
    if (c0 > 0) sg = A.dn[d0 + c0 + (lane < cnt ? lane : cnt - 1)];
    const int32_t total = tri_segs<64>(sg, cnt, lane, L, nullptr);
    wave_sync();
    tri_walk<T, SLOTS, MAXM, MAXS>(A.up_col, L, flg, hq, cnt, 0, total, accw, cntw);
    tri_flush(L, cnt, w0, m, c0 == 0, lane, 64, A.nup, A.Y);
  }
  accw = wave_sum(accw);
  cntw = wave_sum_i64(cntw);
  if (lane == 0) {
    S::store(accw, A.Z, w);
    A.ZT[w] = cntw;
  }
  if (myslot >= 0) L.hkey[myslot] = -1;
}

template <typename T, int SLOTS, int MAXM>
__device__ __forceinline__ void tri_wave_init(TriLds<T, SLOTS, MAXM, 64> &L, int32_t *flg) {
  const int lane = threadIdx.x & 63;
  flg[lane] = 0;
  for (int i = lane; i < SLOTS; i += 64) L.hkey[i] = -1;
  tri_clear_credits(L, lane, 64);
}

// WPB wavefronts per workgroup, each with its own LDS state; the list holds
// the records above: the next node's record is loaded while this one runs,
// and this node's up(w) and first segments are loaded together, so a short
// node waits on one global round trip before its walk.
template <typename T, int SLOTS, int MAXM, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_tri_wave(TriArgs A, const int4 *__restrict__ recs,
                                                        int64_t count) {
  __shared__ TriLds<T, SLOTS, MAXM, 64> lds[WPB];
  __shared__ int32_t flg_s[WPB][kFlg];
  __shared__ int2 hq_s[WPB][kQueue];
  const int wv = threadIdx.x >> 6;
  tri_wave_init(lds[wv], flg_s[wv]);
  const int64_t nwaves = (int64_t)gridDim.x * WPB;
  int64_t it = (int64_t)blockIdx.x * WPB + wv;
  int4 nxt = it < count ? recs[it] : make_int4(0, 0, 0, 0);
  for (; it < count; it += nwaves) {
    const int4 rc = nxt;
    if (it + nwaves < count) nxt = recs[it + nwaves];
    tri_wave_node<T, SLOTS, MAXM>(A, rc, lds[wv], flg_s[wv], hq_s[wv]);
  }
}

// One node w per workgroup of WPB wavefronts sharing one LDS state; chunks
// of MAXS <= NT segments, each wavefront walking a contiguous share of a
// chunk. Every thread calls it (workgroup barriers). On entry flg (each
// wavefront's) is zero and the credit slots are clear (tri_block_init); so
// on return.
template <typename T, int SLOTS, int MAXM, int WPB, int MAXS> struct TriBlockLds {
  TriLds<T, SLOTS, MAXM, MAXS> L;
  int32_t flg[WPB][kFlg];
  int2 hq[WPB][kQueue];
  int32_t part[WPB];
  typename SumT<T>::type acc[WPB];
  int64_t cnt[WPB];
};

template <typename T, int SLOTS, int MAXM, int WPB, int MAXS>
__device__ __forceinline__ void tri_block_init(TriBlockLds<T, SLOTS, MAXM, WPB, MAXS> &B) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (wv < WPB) B.flg[wv][lane] = 0;
  tri_clear_credits(B.L, tid, 64 * WPB);
}

template <typename T, int SLOTS, int MAXM, int WPB, int MAXS>
__device__ __forceinline__ void tri_block_node(const TriArgs &A, int32_t w,
                                               TriBlockLds<T, SLOTS, MAXM, WPB, MAXS> &B) {
  using S = SumT<T>;
  using Acc = typename S::type;
  constexpr int NT = 64 * WPB;
  static_assert(MAXS <= NT, "one segment per thread in the chunk setup");
  auto &L = B.L;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t w0 = A.up_ptr[w], m = A.up_ptr[w + 1] - w0;
  const int32_t d0 = A.dn_ptr[w], nd = A.dn_ptr[w + 1] - d0;
  for (int i = tid; i < SLOTS; i += NT) L.hkey[i] = -1;
  __syncthreads();
  tri_hash<SLOTS, NT>(A.up_col, A.up_deg, w0, m, tid, L.hkey, L.hval);
  Acc accw = Acc();
  int64_t cntw = 0;
  for (int32_t c0 = 0; c0 < nd; c0 += MAXS) {
    const int32_t cnt = nd - c0 < MAXS ? nd - c0 : MAXS;
    const int4 sg = tid < cnt ? A.dn[d0 + c0 + tid] : make_int4(0, 0, 0, 0);
    const int32_t total = tri_segs<NT>(sg, cnt, tid, L, B.part);
    __syncthreads();
    // contiguous shares, multiples of 64 entries
    const int32_t steps = (total + 63) >> 6;
    const int32_t beg = (int32_t)(((int64_t)steps * wv / WPB) << 6);
    const int32_t fin = (int32_t)(((int64_t)steps * (wv + 1) / WPB) << 6);
    tri_walk<T, SLOTS, MAXM, MAXS>(A.up_col, L, B.flg[wv], B.hq[wv], cnt, beg,
                                   fin < total ? fin : total, accw, cntw);
    __syncthreads();
    tri_flush(L, cnt, w0, m, c0 == 0, tid, NT, A.nup, A.Y);
    __syncthreads();
  }
  accw = wave_sum(accw);
  cntw = wave_sum_i64(cntw);
  if (lane == 0) {
    B.acc[wv] = accw;
    B.cnt[wv] = cntw;
  }
  __syncthreads();
  if (tid == 0) {
    Acc a = B.acc[0];
    int64_t cs = B.cnt[0];
    for (int i = 1; i < WPB; ++i) {
      acc_merge(a, B.acc[i]);
      cs += B.cnt[i];
    }
    S::store(a, A.Z, w);
    A.ZT[w] = cs;
  }
  __syncthreads();
}

template <typename T, int SLOTS, int MAXM, int WPB, int MAXS>
__global__ __launch_bounds__(64 * WPB) void k_tri_block(TriArgs A,
                                                         const int32_t *__restrict__ nodes,
                                                         int64_t count) {
  __shared__ TriBlockLds<T, SLOTS, MAXM, WPB, MAXS> B;
  tri_block_init(B);
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x)
    tri_block_node<T, SLOTS, MAXM, WPB, MAXS>(A, nodes[it], B);
}

// |up(w)| too long for LDS: one wavefront per w, one segment per lane, and
// membership by binary search of up(w) (rank order) in global memory.
// Credits to x go to w's upper-end slots with integer atomics (exact, so
// still order-independent; the slots are cleared first), credits to u to the
// lane's own lower-end slot.
template <typename T>
__device__ __forceinline__ void tri_long_node(const TriArgs &A, int32_t w) {
  using S = SumT<T>;
  using Acc = typename S::type;
  const int lane = threadIdx.x & 63;
  const int32_t w0 = A.up_ptr[w], m = A.up_ptr[w + 1] - w0;
  const int32_t d0 = A.dn_ptr[w], nd = A.dn_ptr[w + 1] - d0;
  Acc accw = Acc();
  int64_t cntw = 0;
  for (int32_t base = 0; base < nd; base += 64) {
    const int32_t i = base + lane;
    if (i >= nd) continue;
    const int4 sgm = A.dn[d0 + i];  // {slot of {u, w}, tail length, k_u + k_w, u}
    long long accu = 0;
    int32_t cntu = 0;
    for (int32_t j = sgm.x + 1; j <= sgm.x + sgm.y; ++j) {
      const int32_t x = A.up_col[j], kx = A.up_deg[j];
      int32_t lo = 0, hi = m;  // first member of up(w) not ranked below x
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t y = A.up_col[w0 + mid], ky = A.up_deg[w0 + mid];
        if (ky < kx || (ky == kx && y < x)) lo = mid + 1; else hi = mid;
      }
      if (lo < m && A.up_col[w0 + lo] == x) {
        const T dl = tri_delta<T>(sgm.z + kx);
        const long long f = to_fix(dl);
        S::add_term(accw, dl);
        ++cntw;
        accu += f;
        ++cntu;
        atomicAdd((unsigned long long *)&A.Y[w0 + lo].y, (unsigned long long)f);
        atomicAdd(&A.Y[w0 + lo].t, 1);
      }
    }
    A.Y[A.nup + sgm.x] = TriSlot{accu, cntu, 0};
  }
  accw = wave_sum(accw);
  cntw = wave_sum_i64(cntw);
  if (lane == 0) {
    S::store(accw, A.Z, w);
    A.ZT[w] = cntw;
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_tri_long(TriArgs A, const int32_t *__restrict__ nodes,
                                                 int64_t count) {
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) tri_long_node<T>(A, nodes[it]);
}

// One node w per lane (|up(w)| <= M, a walk of at most kTriLaneWork entries),
// for the many nodes whose whole triangle work is a few membership tests: a
// wavefront per node would spend its time on setup. up(w) sits in registers
// (a test compares against all M entries), the credits to x by position and
// to u by segment in per-lane integer slots (the LDS slots' representation,
// so the records are the same bits as the other bins would write). Nodes are
// listed by id, so neighbouring lanes read neighbouring rows.
template <typename T> struct LaneSlot;
template <> struct LaneSlot<float> {
  unsigned long long w = 0;
  __device__ void add(float dl) {
    w += (1ull << 44) + (unsigned long long)(uint32_t)(-dl * 16777216.0f);
  }
  __device__ TriSlot slot() const {
    return TriSlot{-(long long)((w & ((1ull << 44) - 1)) << 12), (int32_t)(w >> 44), 0};
  }
};
template <> struct LaneSlot<double> {
  long long y = 0;
  int32_t t = 0;
  __device__ void add(double dl) {
    y += to_fix(dl);
    ++t;
  }
  __device__ TriSlot slot() const { return TriSlot{y, t, 0}; }
};
template <> struct LaneSlot<TriCount> {
  int32_t t = 0;
  __device__ void add(TriCount) { ++t; }
  __device__ TriSlot slot() const { return TriSlot{0, t, 0}; }
};

template <typename T, int M>
__device__ __forceinline__ void tri_lane_node(const TriArgs &A, const int4 rc) {
  using S = SumT<T>;
  using Acc = typename S::type;
  const int32_t w = rc.x, w0 = rc.y, d0 = rc.z;
  const int32_t m = rc.w & 0xFF, nd = (rc.w >> 8) & 0xFF, walk = rc.w >> 16;
  int32_t up[M];
#pragma unroll
  for (int q = 0; q < M; ++q) up[q] = q < m ? A.up_col[w0 + q] : -1;
  LaneSlot<T> acc[M];
  LaneSlot<T> su;
  Acc accw = Acc();
  int64_t cntw = 0;
  // every listed node has nd >= 1 segments, each non-empty; walk = their total
  int32_t s = 0;
  int4 sg = A.dn[d0];
  int32_t j = sg.x + 1, jend = sg.x + sg.y;
  for (int32_t t = 0; t < walk; ++t) {
    const int32_t x = A.up_col[j], kx = A.up_deg[j];
    int32_t p = -1;
#pragma unroll
    for (int q = 0; q < M; ++q) p = up[q] == x ? q : p;
    if (p >= 0) {
      const T dl = tri_delta<T>(sg.z + kx);
      S::add_term(accw, dl);
      ++cntw;
      su.add(dl);
#pragma unroll
      for (int q = 0; q < M; ++q)
        if (q == p) acc[q].add(dl);
    }
    if (++j > jend) {
      A.Y[A.nup + sg.x] = su.slot();
      su = LaneSlot<T>();
      if (++s < nd) {
        sg = A.dn[d0 + s];
        j = sg.x + 1;
        jend = sg.x + sg.y;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < M; ++q)
    if (q < m) A.Y[w0 + q] = acc[q].slot();
  S::store(accw, A.Z, w);
  A.ZT[w] = cntw;
}

template <typename T, int M>
__global__ __launch_bounds__(256) void k_tri_lane(TriArgs A, const int4 *__restrict__ recs,
                                                  int64_t count) {
  for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < count;
       it += (int64_t)gridDim.x * blockDim.x)
    tri_lane_node<T, M>(A, recs[it]);
}

// Clear the listed records (upper-end records of long-list nodes, which
// their walk adds to with atomics). Records no walk writes are never read:
// readers skip trec = -1, and read Z / ZT only of nodes with segments.
__global__ void k_tri_zero(TriSlot *__restrict__ Y, const int32_t *__restrict__ zl, int64_t nz) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nz;
       i += (int64_t)gridDim.x * blockDim.x)
    Y[zl[i]] = TriSlot{0, 0, 0};
}

static unsigned cap_blocks_tri(int64_t b, int64_t cap) {
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

// node lists: see kTriBin* (wavefront, 8-wavefront and 16-wavefront
// workgroups, long lists)
template <typename T>
static hipError_t tri_impl(const Graph &g, TriSlot *Y, void *Z, int64_t *ZT, hipStream_t st) {
  const TriArgs A{g.up_ptr, g.up_col, g.up_deg, g.dn_ptr, g.dn, g.nnz / 2, Y, Z, ZT};
  if (g.n_tri_zero > 0)
    hipLaunchKernelGGL(k_tri_zero, dim3(cap_blocks_tri((g.n_tri_zero + 255) / 256, 1 << 16)),
                       dim3(256), 0, st, Y, g.tri_zero, g.n_tri_zero);
  const int64_t *counts = g.n_tri;
  if (g.n_tri_lane > 0)
    hipLaunchKernelGGL((k_tri_lane<T, kTriLaneM>),
                       dim3(cap_blocks_tri((g.n_tri_lane + 255) / 256, 1 << 16)), dim3(256), 0, st,
                       A, g.tri_recL, g.n_tri_lane);
  if (counts[0] > 0)
    hipLaunchKernelGGL((k_tri_wave<T, 256, 64, 4>), dim3(cap_blocks_tri((counts[0] + 3) / 4, 1 << 20)),
                       dim3(256), 0, st, A, g.tri_rec0, counts[0]);
  if (counts[1] > 0)
    hipLaunchKernelGGL((k_tri_block<T, 2048, 512, 8, 512>), dim3(cap_blocks_tri(counts[1], 1 << 20)),
                       dim3(512), 0, st, A, g.tri_list[1], counts[1]);
  if (counts[2] > 0)
    hipLaunchKernelGGL((k_tri_block<T, 8192, 2048, 16, 1024>),
                       dim3(cap_blocks_tri(counts[2], 1 << 20)), dim3(1024), 0, st, A, g.tri_list[2],
                       counts[2]);
  if (counts[3] > 0)
    hipLaunchKernelGGL(k_tri_long<T>, dim3(cap_blocks_tri(counts[3], 1 << 20)), dim3(64), 0, st, A,
                       g.tri_list[3], counts[3]);
  return hipGetLastError();
}

hipError_t launch_triangles_count(const Graph &g, TriSlot *Y, int64_t *ZT, hipStream_t st) {
  return tri_impl<TriCount>(g, Y, nullptr, ZT, st);
}

hipError_t launch_triangles(const Graph &g, ef_prec prec, TriSlot *Y, void *Z, int64_t *ZT,
                            hipStream_t st) {
  if (prec == EF_PREC_FP64) return tri_impl<double>(g, Y, Z, ZT, st);
  return tri_impl<float>(g, Y, Z, ZT, st);
}

}  // namespace efi
