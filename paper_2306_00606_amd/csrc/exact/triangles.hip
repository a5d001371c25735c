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
#include <type_traits>

#include "device_common.h"

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

// In FP32C the credit of w (the middle node) is the sum of the credits of
// the x's: it is taken from the exact x slots when they are flushed, instead
// of a compensated sum per hit.
template <typename T> constexpr bool kZFromSlots = std::is_same<T, float>::value;
__device__ __forceinline__ DFv dfv_from_fix(long long y) {
  const double d = (double)y * (1.0 / kTriFix);
  DFv r;
  r.hi = (float)d;
  r.lo = (float)(d - (double)r.hi);
  return r;
}

// LDS hash set of up(w) for the walk: linear probing on single-word keys
// (empty = -1), with slot SLOTS mirroring slot 0 in both arrays so a lookup
// reads its first two slots with one two-word LDS read and no wrap. Home:
// the 24-bit multiplicative hash of the id's low 24 bits (ids that agree
// there share a home; lookups stay exact).
template <int SLOTS> struct TriHash {
  static_assert(SLOTS >= 2 && (SLOTS & (SLOTS - 1)) == 0, "SLOTS must be a power of two");
  static constexpr int kBits = __builtin_ctz(SLOTS);
  __device__ static __forceinline__ uint32_t home(int32_t x) {
    // 24-bit operands: one v_mul_u32_u24, unsigned shift
    return (((uint32_t)x & 0xFFFFFFu) * 0x9E3779u) >> (32 - kBits);
  }
  // x not yet in the set; stores x and its value v, returns the slot
  __device__ static __forceinline__ int32_t insert(int32_t *keys, int32_t *vals, int32_t x,
                                                   int32_t v) {
    uint32_t h = home(x);
    while (atomicCAS(&keys[h], -1, x) != -1) h = (h + 1) & (SLOTS - 1);
    vals[h] = v;
    if (h == 0) {
      keys[SLOTS] = x;
      vals[SLOTS] = v;
    }
    return (int32_t)h;
  }
  __device__ static __forceinline__ void erase(int32_t *keys, int32_t slot) {
    keys[slot] = -1;
    if (slot == 0) keys[SLOTS] = -1;
  }
  // a lookup in two parts, so several can have their first read in flight:
  // probe() reads the first two slots of x's run, resolve() returns the slot
  // of x (SLOTS for slot 0 reached as the second probe) or -1
  __device__ static __forceinline__ int2 probe(const int32_t *keys, uint32_t h) {
    return make_int2(keys[h], keys[h + 1]);
  }
  __device__ static __forceinline__ int32_t resolve(const int32_t *keys, int32_t x, uint32_t h,
                                                    int2 ab) {
    int32_t slot = ab.x == x ? (int32_t)h : (ab.x != -1 && ab.y == x) ? (int32_t)h + 1 : -1;
    if (ab.x != x && ab.x != -1 && ab.y != x && ab.y != -1) {
      uint32_t p = (h + 2) & (SLOTS - 1);
      int32_t k;
      while ((k = keys[p]) != x && k != -1) p = (p + 1) & (SLOTS - 1);
      slot = k == x ? (int32_t)p : -1;
    }
    return slot;
  }
};

// LDS state of one w:
//   hkey[SLOTS+1] ids x of up(w) (TriHash), hval[slot] = k_x << kPosBits |
//                 position of x in up(w)
//   seg[MAXS]     per segment of the chunk: {4 x (first index of the tail in
//                 up_col minus its first index in the concatenated sequence),
//                 (k_u + k_w) << 11 | segment}
//   segp[MAXS+1]  first concatenated index of each segment; segp[nseg] = total
//   acc, cnt      credits to x by position in up(w)
//   sacc, scnt    credits to u by segment, u_copies<MAXS>() slots per segment
//                 (by lane parity: the hits of one segment arrive in runs,
//                 and adds to one LDS address serialise)
constexpr int kSegBits = 11;
// credit slots per segment: 4 in the workgroup bins (long runs of hits per
// segment), 1 in the wavefront bins (short runs; LDS decides occupancy there)
template <int MAXS> constexpr int u_copies() { return MAXS <= 64 ? 1 : 4; }
static_assert(kMaxDegree < (1u << 20), "k_u + k_w must fit above the segment field");
template <typename T, int SLOTS, int MAXM, int MAXS> struct TriLds {
  static_assert(SLOTS >= 2 * MAXM, "the hash set of up(w) must stay at most half full");
  static_assert(MAXM <= (1 << 11) && MAXS <= (1 << kSegBits),
                "credit slots hold at most 2^11 credits; segment field");
  __align__(16) int32_t hkey[SLOTS + 4];
  int32_t hval[SLOTS + 4];
  int2 seg[MAXS];
  int32_t segp[MAXS + 1];
  unsigned long long acc[MAXM];
  static constexpr int kUCopies = u_copies<MAXS>();
  unsigned long long sacc[MAXS * kUCopies];
  int32_t cnt[Credit<T>::kPacked ? 1 : MAXM];
  int32_t scnt[Credit<T>::kPacked ? 1 : MAXS * kUCopies];
};

// Hash up(w) (m entries from w0) with NT threads; returns the slot this
// thread filled last (-1 if none).
template <int SLOTS, int NT>
__device__ __forceinline__ int32_t tri_hash(const int32_t *__restrict__ up_col,
                                            const int32_t *__restrict__ up_deg, int32_t w0,
                                            int32_t m, int tid, int32_t *hkey, int32_t *hval) {
  int32_t myslot = -1;
  for (int32_t i = tid; i < m; i += NT)
    myslot = TriHash<SLOTS>::insert(hkey, hval, up_col[w0 + i], pack_kp(up_deg[w0 + i], i));
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
    lds.seg[tid] = make_int2(4 * (e.x + 1 - start), (e.z << kSegBits) | tid);
    lds.segp[tid] = start;
  }
  if (tid == 0) lds.segp[cnt] = total;
  return total;
}

// One wavefront walks entries [beg, end) of the chunk's concatenated tails,
// 64 consecutive entries per step. A hit (x in up(w)) is appended to the
// wavefront's LDS queue as two words, {sigma, segment | pos(x) << 16};
// whenever 64 hits are queued they are scored and credited with every lane
// busy, so the hit path does not run divergently on almost every step.
constexpr int kQueue = 128;
// tri_walk drains once the queue holds 64 hits, so up to 63 wait while a
// wavefront appends up to 64 more: indices reach 126
static_assert(kQueue >= 127, "the hit queue must hold 63 waiting + 64 new hits");

// Segment of each lane's entry. Tails are long (tens to hundreds of
// entries), so most steps lie inside one segment or cross one to three
// segment starts. Once per 64 steps, each lane finds by binary search the
// segment holding the first entry of one step and packs it with the starts
// of the next three segments relative to the step (step word: segment in
// bits 0-10, starts in bits 11-17, 18-24, 25-31; 64 and above: no start in
// the step; 0 in the last field: four or more starts). A step then takes
// its word from that lane and compares each lane with at most three
// starts; a step with more starts flags them in LDS and reads them back as
// a ballot (flg: 64 words of scratch, cleared before each use).
__device__ __forceinline__ int32_t lanes_below(unsigned long long m) {
  return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// word of the step at c (< total) of a chunk with nseg segments
__device__ __forceinline__ int32_t step_word(const int32_t *segp, int32_t nseg, int32_t c) {
  const int32_t s0 = seg_find(segp, nseg, c);
  int32_t w = s0;
#pragma unroll
  for (int k = 1; k <= 3; ++k) {
    const int32_t b = s0 + k < nseg ? segp[s0 + k] - c : 127;
    w |= (b < 127 ? b : 127) << (4 + 7 * k);
  }
  if (s0 + 4 < nseg && segp[s0 + 4] < c + 64) w &= 0x01FFFFFF;  // four or more starts
  return w;
}

// segment of entry c + lane (every lane: entries at or past the total get
// the last segment, whose start is the last one counted) from the step word
__device__ __forceinline__ int32_t step_seg(const int32_t *segp, int32_t nseg, int32_t c,
                                            int32_t w, int32_t *flg) {
  const int32_t lane = (int32_t)(threadIdx.x & 63);
  const int32_t s0 = w & 0x7FF;
  const int32_t b1 = (w >> 11) & 127, b2 = (w >> 18) & 127, b3 = (int32_t)((uint32_t)w >> 25);
  if (b1 >= 64) return s0;  // inside one segment (most steps)
  if (b2 >= 64) return s0 + (lane >= b1 ? 1 : 0);
  if (b3 != 0) return s0 + (lane >= b1 ? 1 : 0) + (lane >= b2 ? 1 : 0) + (lane >= b3 ? 1 : 0);
  const int32_t s = s0 + 1 + lane;
  const int32_t vb = s < nseg ? segp[s] : INT32_MAX;
  const bool in = vb < c + 64;
  wave_sync();
  flg[lane] = 0;
  wave_sync();
  if (in) flg[vb - c] = 1;
  wave_sync();
  const int32_t f = flg[lane];
  const unsigned long long starts = __builtin_amdgcn_ballot_w64(f != 0);
  return s0 + lanes_below(starts) + (f != 0);
}

// One round of U steps at c, c + 64, ...: the member x of entry c + lane and
// its segment word ((k_u + k_w) << 11 | segment). Lanes at or past the total
// load its last entry, steps past the block the last entry: every load is
// valid and unconditional, so a round's loads stay in flight across the
// previous round's work; the use masks lanes at or past end. The segments
// of all U steps are found first (seg_of(step, c)), then their LDS reads
// and global loads are issued together. jn steps in the block, j the
// round's first step. Loads address up_col by 32-bit byte offsets (the
// segment table holds 4 x its element offsets; up_col has fewer than 2^29
// entries).
template <int U, typename L, typename SegOf>
__device__ __forceinline__ void tri_fetch(const int32_t *__restrict__ up_col, const L &lds,
                                          int32_t nseg, int32_t total, int32_t c, int32_t j,
                                          int32_t jn, SegOf seg_of, int32_t (&x)[U],
                                          int32_t (&sy)[U]) {
  const int32_t lane4 = (int32_t)(threadIdx.x & 63) * 4;
  int32_t sg[U], boff[U];
  if (j + U <= jn && c + 64 * U <= total) {
    // (most rounds) every step in the block and inside the chunk
#pragma unroll
    for (int q = 0; q < U; ++q) {
      sg[q] = seg_of(j + q, c + 64 * q);
      boff[q] = 4 * (c + 64 * q) + lane4;
    }
  } else {
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int32_t cq = c + 64 * q;
      sg[q] = nseg - 1;
      boff[q] = 4 * (total - 1);
      if (j + q < jn) {
        sg[q] = seg_of(j + q, cq);
        boff[q] = 4 * min(cq + lane4 / 4, total - 1);
      }
    }
  }
  int2 sv[U];
#pragma unroll
  for (int q = 0; q < U; ++q) sv[q] = lds.seg[sg[q]];
  const char *base = reinterpret_cast<const char *>(up_col);
#pragma unroll
  for (int q = 0; q < U; ++q) {
    x[q] = *reinterpret_cast<const int32_t *>(base + (uint32_t)(sv[q].x + boff[q]));
    sy[q] = sv[q].y;
  }
}

template <typename T, int SLOTS, int MAXM, int MAXS>
__device__ __forceinline__ void tri_walk(const int32_t *__restrict__ up_col,
                                         TriLds<T, SLOTS, MAXM, MAXS> &L, int2 *hq,
                                         int32_t nseg, int32_t beg, int32_t end,
                                         typename SumT<T>::type &accw, int64_t &cntw) {
  using S = SumT<T>;
  constexpr int32_t kPosMask = (1 << kPosBits) - 1;
  // short walks (wavefront bins: a few steps per node) waste less with two
  constexpr int U = MAXS <= 64 ? 2 : 4;
  beg = __builtin_amdgcn_readfirstlane(beg);
  end = __builtin_amdgcn_readfirstlane(end);
  nseg = __builtin_amdgcn_readfirstlane(nseg);
  if (beg >= end) return;
  const int lane = threadIdx.x & 63;
  const char *hkey = reinterpret_cast<const char *>(L.hkey);
  const char *hval = reinterpret_cast<const char *>(L.hval);
  const int32_t total = __builtin_amdgcn_readfirstlane(L.segp[nseg]);
  // the flags of steps with many segment starts use the queue's last 32
  // entries: segments are found before a round's hits are appended, when at
  // most 63 hits wait
  int32_t *const flg = reinterpret_cast<int32_t *>(hq + (kQueue - 32));
  int32_t qn = 0;  // queued hits (uniform)
  // score and credit hq[qn - cnt .. qn) on lanes 0 .. cnt-1; a queued hit is
  // {segment word, hval of x}
  auto drain = [&](int32_t cnt) {
    wave_sync();
    if (lane < cnt) {
      const int2 h = hq[qn - cnt + lane];
      const T dl = tri_delta<T>((h.x >> kSegBits) + unpack_k(h.y));
      if constexpr (!kZFromSlots<T>) S::add_term(accw, dl);
      Credit<T>::add(L.acc, L.cnt, h.y & kPosMask, dl);
      constexpr int K = u_copies<MAXS>();
      Credit<T>::add(L.sacc, L.scnt, (h.x & ((1 << kSegBits) - 1)) * K + (lane & (K - 1)), dl);
    }
    cntw += cnt;
    qn -= cnt;
    wave_sync();
  };
  // a round: the U probes first (the first two slots of each x's run in one
  // two-word read, byte offsets throughout), then the values of the hits,
  // then the appends (and drains) step by step. Hits are kept as wavefront
  // lane masks (scalar registers) and turned back into lane predicates with
  // inverse ballots.
  auto use = [&](const int32_t (&x)[U], const int32_t (&sy)[U], int32_t c) {
    uint32_t h4[U];
    int2 ab[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      h4[q] = TriHash<SLOTS>::home(x[q]) << 2;
      const int32_t *p = reinterpret_cast<const int32_t *>(hkey + h4[q]);
      ab[q] = make_int2(p[0], p[1]);
    }
    unsigned long long hm[U];
    uint32_t s4[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const unsigned long long fa = __builtin_amdgcn_ballot_w64(ab[q].x == x[q]);
      const unsigned long long ea = __builtin_amdgcn_ballot_w64(ab[q].x == -1);
      const unsigned long long fb = __builtin_amdgcn_ballot_w64(ab[q].y == x[q]);
      const unsigned long long eb = __builtin_amdgcn_ballot_w64(ab[q].y == -1);
      hm[q] = fa | (fb & ~ea);
      s4[q] = h4[q] + (__builtin_amdgcn_inverse_ballot_w64(fa) ? 0u : 4u);
      const unsigned long long more = ~(fa | ea | fb | eb);
      if (more != 0ull) {
        // rare: the run continues past its first two slots. The outcome is
        // a slot value (kNoSlot: absent) and its ballot is taken once every
        // lane has left the loop.
        constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
        uint32_t r = s4[q];
        if (__builtin_amdgcn_inverse_ballot_w64(more)) {
          uint32_t pp = (h4[q] + 8) & (4 * SLOTS - 4);
          int32_t k;
          while ((k = *reinterpret_cast<const int32_t *>(hkey + pp)) != x[q] && k != -1)
            pp = (pp + 4) & (4 * SLOTS - 4);
          r = k == x[q] ? pp : kNoSlot;
        }
        hm[q] |= __builtin_amdgcn_ballot_w64(r != kNoSlot) & more;
        s4[q] = r;
      }
      // lanes at or past end (whole steps past it in the last round)
    }
    if (end - c < 64 * U) {
      // the last round: lanes at or past end (whole steps past it)
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int32_t left = end - (c + 64 * q);
        if (left < 64) hm[q] &= left > 0 ? (1ull << left) - 1ull : 0ull;
      }
    }
    int32_t ev[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      ev[q] = 0;
      if (__builtin_amdgcn_inverse_ballot_w64(hm[q]))
        ev[q] = *reinterpret_cast<const int32_t *>(hval + s4[q]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (__builtin_amdgcn_inverse_ballot_w64(hm[q]))
        hq[qn + lanes_below(hm[q])] = make_int2(sy[q], ev[q]);
      qn += __popcll(hm[q]);
      if (qn >= 64) drain(64);
    }
  };
  // two rounds in flight: round r + 1 is fetched before round r is used, so
  // its loads overlap the hash probes and drains of round r
  auto rounds = [&](int32_t cb, int32_t jn, auto seg_of) {
    int32_t xa[U], ya[U], xb[U], yb[U];
    tri_fetch<U>(up_col, L, nseg, total, cb, 0, jn, seg_of, xa, ya);
    for (int32_t j = 0;;) {
      tri_fetch<U>(up_col, L, nseg, total, cb + 64 * (j + U), j + U, jn, seg_of, xb, yb);
      use(xa, ya, cb + 64 * j);
      j += U;
      if (j >= jn) break;
      tri_fetch<U>(up_col, L, nseg, total, cb + 64 * (j + U), j + U, jn, seg_of, xa, ya);
      use(xb, yb, cb + 64 * j);
      j += U;
      if (j >= jn) break;
    }
  };
  const int32_t nsteps = (end - beg + 63) >> 6;
  if constexpr (MAXS <= 64) {
    // at most 64 segments: their starts sit in one register (lane s: start
    // of segment s), and a step's segments come from ballots over it
    const int32_t segv = lane < nseg ? L.segp[lane] : INT32_MAX;
    rounds(beg, nsteps, [&](int32_t, int32_t c) {
      const int32_t s0 = __popcll(__builtin_amdgcn_ballot_w64(segv <= c)) - 1;
      const bool in = segv > c && segv < c + 64;
      const unsigned long long m_in = __builtin_amdgcn_ballot_w64(in);
      int32_t sg = s0;
      if (m_in == 0ull) return sg;
      if (__popcll(m_in) <= 3) {
        unsigned long long m = m_in;
        while (m != 0ull) {
          const int j = __builtin_ctzll(m);
          m &= m - 1ull;
          sg += (c + lane >= __builtin_amdgcn_readlane(segv, j)) ? 1 : 0;
        }
      } else {
        wave_sync();
        flg[lane] = 0;
        wave_sync();
        if (in) flg[segv - c] = 1;
        wave_sync();
        const int32_t f = flg[lane];
        const unsigned long long starts = __builtin_amdgcn_ballot_w64(f != 0);
        sg += lanes_below(starts) + (f != 0);
      }
      return sg;
    });
  } else {
    for (int32_t jb = 0; jb < nsteps; jb += 64) {
      const int32_t cb = beg + 64 * jb;
      const int32_t jn = nsteps - jb < 64 ? nsteps - jb : 64;
      const int32_t win = lane < jn ? step_word(L.segp, nseg, cb + 64 * lane) : 0;
      rounds(cb, jn, [&](int32_t j, int32_t c) {
        return step_seg(L.segp, nseg, c, __builtin_amdgcn_readlane(win, j), flg);
      });
    }
  }
  wave_sync();
  if (qn > 0) drain(qn);
}

// After a chunk: the credits to u go to the segments' lower-end slots, the
// credits to x are stored (first chunk) or added to w's upper-end slots, and
// the x credits this thread flushed are added to zs (2^-36 units). Clears
// both for the next chunk.
template <typename T, int SLOTS, int MAXM, int MAXS>
__device__ __forceinline__ void tri_flush(TriLds<T, SLOTS, MAXM, MAXS> &L, int32_t cnt, int32_t w0,
                                          int32_t m, bool first, int tid, int nt, int64_t nup,
                                          TriSlot *Y, long long &zs) {
  constexpr int kUCopies = u_copies<MAXS>();
  for (int32_t i = tid; i < cnt; i += nt) {
    TriSlot r{0, 0, 0};
#pragma unroll
    for (int k = 0; k < kUCopies; ++k) {
      long long y;
      int32_t t;
      Credit<T>::load(L.sacc, L.scnt, i * kUCopies + k, y, t);
      r.y += y;
      r.t += t;
      L.sacc[i * kUCopies + k] = 0ull;
      if constexpr (!Credit<T>::kPacked) L.scnt[i * kUCopies + k] = 0;
    }
    // slot of {u, w} in up(u): the entry before the tail
    Y[nup + (L.seg[i].x >> 2) + L.segp[i] - 1] = r;
  }
  for (int32_t i = tid; i < m; i += nt) {
    TriSlot r{0, 0, 0};
    Credit<T>::load(L.acc, L.cnt, i, r.y, r.t);
    zs += r.y;
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
  for (int i = tid; i < MAXS * u_copies<MAXS>(); i += nt) {
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
// segment, |up(w)| | segments << 16}. On entry the hash holds no key and the
// credit slots are clear (tri_wave_init); on return too: each
// lane empties the one hash slot it filled, so a short list does not pay for
// the whole table.
template <typename T, int SLOTS, int MAXM>
__device__ __forceinline__ void tri_wave_node(const TriArgs &A, const int4 rc,
                                              TriLds<T, SLOTS, MAXM, 64> &L, int2 *hq) {
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
  if (lane < m) myslot = TriHash<SLOTS>::insert(L.hkey, L.hval, x, pack_kp(kx, lane));
  Acc accw = Acc();
  int64_t cntw = 0;
  long long zs = 0;
  for (int32_t c0 = 0; c0 < nd; c0 += MAXS) {
    const int32_t cnt = nd - c0 < MAXS ? nd - c0 : MAXS;
    if (c0 > 0) sg = A.dn[d0 + c0 + (lane < cnt ? lane : cnt - 1)];
    const int32_t total = tri_segs<64>(sg, cnt, lane, L, nullptr);
    wave_sync();
    tri_walk<T, SLOTS, MAXM, MAXS>(A.up_col, L, hq, cnt, 0, total, accw, cntw);
    tri_flush(L, cnt, w0, m, c0 == 0, lane, 64, A.nup, A.Y, zs);
  }
  if constexpr (kZFromSlots<T>) accw = dfv_from_fix(wave_sum_i64(zs));
  else accw = wave_sum(accw);
  if (lane == 0) {
    S::store(accw, A.Z, w);
    A.ZT[w] = cntw;  // the walk counts hits per wavefront
  }
  if (myslot >= 0) TriHash<SLOTS>::erase(L.hkey, myslot);
}

template <typename T, int SLOTS, int MAXM>
__device__ __forceinline__ void tri_wave_init(TriLds<T, SLOTS, MAXM, 64> &L) {
  const int lane = threadIdx.x & 63;
  for (int i = lane; i <= SLOTS; i += 64) L.hkey[i] = -1;
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
  __shared__ int2 hq_s[WPB][kQueue];
  const int wv = threadIdx.x >> 6;
  tri_wave_init(lds[wv]);
  const int64_t nwaves = (int64_t)gridDim.x * WPB;
  int64_t it = (int64_t)blockIdx.x * WPB + wv;
  int4 nxt = it < count ? recs[it] : make_int4(0, 0, 0, 0);
  for (; it < count; it += nwaves) {
    const int4 rc = nxt;
    if (it + nwaves < count) nxt = recs[it + nwaves];
    tri_wave_node<T, SLOTS, MAXM>(A, rc, lds[wv], hq_s[wv]);
  }
}

// One node w per workgroup of WPB wavefronts sharing one LDS state; chunks
// of MAXS <= NT segments, each wavefront walking a contiguous share of a
// chunk. Every thread calls it (workgroup barriers). rc = {w, first up slot,
// first segment, |up(w)| | segments << 12}. On entry the hash holds no key
// and the credit slots are clear (tri_block_init); so on return: each
// thread empties the hash slots it filled.
template <typename T, int SLOTS, int MAXM, int WPB, int MAXS> struct TriBlockLds {
  TriLds<T, SLOTS, MAXM, MAXS> L;
  int2 hq[WPB][kQueue];
  int32_t part[WPB];
  typename SumT<T>::type acc[WPB];
  int64_t cnt[WPB];
  long long zs[WPB];
};

template <typename T, int SLOTS, int MAXM, int WPB, int MAXS>
__device__ __forceinline__ void tri_block_init(TriBlockLds<T, SLOTS, MAXM, WPB, MAXS> &B) {
  const int tid = threadIdx.x;
  for (int i = tid; i <= SLOTS; i += 64 * WPB) B.L.hkey[i] = -1;
  tri_clear_credits(B.L, tid, 64 * WPB);
  __syncthreads();
}

// next: the record of the node this workgroup takes after rc (or null),
// loaded into nrc together with rc's up(w) and first segments, so a node
// waits on one global round trip before its walk
template <typename T, int SLOTS, int MAXM, int WPB, int MAXS>
__device__ __forceinline__ void tri_block_node(const TriArgs &A, const int4 rc,
                                               TriBlockLds<T, SLOTS, MAXM, WPB, MAXS> &B,
                                               const int4 *next, int4 &nrc) {
  using S = SumT<T>;
  using Acc = typename S::type;
  constexpr int NT = 64 * WPB;
  constexpr int R = (MAXM + NT - 1) / NT;  // up(w) entries per thread
  static_assert(MAXS <= NT, "one segment per thread in the chunk setup");
  auto &L = B.L;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t w = rc.x, w0 = rc.y, d0 = rc.z, m = rc.w & 0xFFF, nd = rc.w >> 12;
  int32_t xs[R], ks[R], slots[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int32_t i = tid + r * NT;
    xs[r] = i < m ? A.up_col[w0 + i] : 0;
    ks[r] = i < m ? A.up_deg[w0 + i] : 0;
  }
  int4 sg = tid < nd && tid < MAXS ? A.dn[d0 + tid] : make_int4(0, 0, 0, 0);
  if (next) nrc = *next;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int32_t i = tid + r * NT;
    slots[r] = i < m ? TriHash<SLOTS>::insert(L.hkey, L.hval, xs[r], pack_kp(ks[r], i)) : -1;
  }
  Acc accw = Acc();
  int64_t cntw = 0;
  long long zs = 0;
  for (int32_t c0 = 0; c0 < nd; c0 += MAXS) {
    const int32_t cnt = nd - c0 < MAXS ? nd - c0 : MAXS;
    if (c0 > 0) sg = tid < cnt ? A.dn[d0 + c0 + tid] : make_int4(0, 0, 0, 0);
    // (the scan's barriers also publish the hash inserts)
    const int32_t total = tri_segs<NT>(sg, cnt, tid, L, B.part);
    __syncthreads();
    // contiguous shares, multiples of 64 entries
    const int32_t steps = (total + 63) >> 6;
    const int32_t beg = (int32_t)(((int64_t)steps * wv / WPB) << 6);
    const int32_t fin = (int32_t)(((int64_t)steps * (wv + 1) / WPB) << 6);
    tri_walk<T, SLOTS, MAXM, MAXS>(A.up_col, L, B.hq[wv], cnt, beg,
                                   fin < total ? fin : total, accw, cntw);
    __syncthreads();
    tri_flush(L, cnt, w0, m, c0 == 0, tid, NT, A.nup, A.Y, zs);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (slots[r] >= 0) TriHash<SLOTS>::erase(L.hkey, slots[r]);
  if constexpr (kZFromSlots<T>) zs = wave_sum_i64(zs);
  else accw = wave_sum(accw);
  if (lane == 0) {
    B.acc[wv] = accw;
    B.zs[wv] = zs;
    B.cnt[wv] = cntw;  // the walk counts hits per wavefront
  }
  __syncthreads();
  if (tid == 0) {
    Acc a = B.acc[0];
    long long z = B.zs[0];
    int64_t cs = B.cnt[0];
    for (int i = 1; i < WPB; ++i) {
      acc_merge(a, B.acc[i]);
      z += B.zs[i];
      cs += B.cnt[i];
    }
    if constexpr (kZFromSlots<T>) a = dfv_from_fix(z);
    S::store(a, A.Z, w);
    A.ZT[w] = cs;
  }
  __syncthreads();
}

// the same for a node given by id (its record built from the row pointers)
template <typename T, int SLOTS, int MAXM, int WPB, int MAXS>
__device__ __forceinline__ void tri_block_node(const TriArgs &A, int32_t w,
                                               TriBlockLds<T, SLOTS, MAXM, WPB, MAXS> &B) {
  const int32_t w0 = A.up_ptr[w], d0 = A.dn_ptr[w];
  const int4 rc = make_int4(w, w0, d0, (A.up_ptr[w + 1] - w0) | ((A.dn_ptr[w + 1] - d0) << 12));
  int4 unused;
  tri_block_node<T, SLOTS, MAXM, WPB, MAXS>(A, rc, B, nullptr, unused);
}

template <typename T, int SLOTS, int MAXM, int WPB, int MAXS, int WPE>
__global__ __launch_bounds__(64 * WPB, WPE) void k_tri_block(TriArgs A,
                                                              const int4 *__restrict__ recs,
                                                              int64_t count) {
  __shared__ TriBlockLds<T, SLOTS, MAXM, WPB, MAXS> B;
  tri_block_init(B);
  int64_t it = blockIdx.x;
  if (it >= count) return;
  int4 rc = recs[it];
  for (; it < count; it += gridDim.x) {
    const int64_t nx = it + gridDim.x;
    int4 nrc = rc;
    tri_block_node<T, SLOTS, MAXM, WPB, MAXS>(A, rc, B, nx < count ? recs + nx : nullptr, nrc);
    rc = nrc;
  }
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
    hipLaunchKernelGGL((k_tri_block<T, 2048, 512, 8, 512, 6>), dim3(cap_blocks_tri(counts[1], 1 << 20)),
                       dim3(512), 0, st, A, g.tri_recB[1], counts[1]);
  if (counts[2] > 0)
    hipLaunchKernelGGL((k_tri_block<T, 4096, 2048, 16, 1024, 4>),
                       dim3(cap_blocks_tri(counts[2], 1 << 20)), dim3(1024), 0, st, A, g.tri_recB[2],
                       counts[2]);
  if (counts[3] > 0)
    hipLaunchKernelGGL(k_tri_long<T>, dim3(cap_blocks_tri(counts[3], 1 << 20)), dim3(64), 0, st, A,
                       g.tri_list[3], counts[3]);
  return hipGetLastError();
}

hipError_t launch_triangles(const Graph &g, ef_prec prec, TriSlot *Y, void *Z, int64_t *ZT,
                            hipStream_t st) {
  if (prec == EF_PREC_FP64) return tri_impl<double>(g, Y, Z, ZT, st);
  return tri_impl<float>(g, Y, Z, ZT, st);
}

}  // namespace efi
