// Device helpers shared by the kernel translation units.
#pragma once

#include "ef_internal.h"

namespace efi {

__device__ __forceinline__ bool rank_less_d(int32_t a, int32_t ka, int32_t b, int32_t kb) {
  return ka < kb || (ka == kb && a < b);
}

// double-float accumulator (FP32 path)
struct DFv {
  float hi, lo;
  __device__ __forceinline__ void add(float x) {
    float s = hi + x;
    float bb = s - hi;
    float e = (hi - (s - bb)) + (x - bb);
    hi = s;
    lo += e;
  }
  __device__ __forceinline__ void add(DFv o) {
    add(o.hi);
    add(o.lo);
  }
  __device__ __forceinline__ double value() const { return (double)hi + (double)lo; }
};

template <typename T> struct SumT;
template <> struct SumT<float> {
  using type = DFv;
  __device__ static void add_stored(DFv &a, const void *p, int64_t i) {
    float2 x = reinterpret_cast<const float2 *>(p)[i];
    a.add(x.x);
    a.add(x.y);
  }
  __device__ static void store(const DFv &a, void *p, int64_t i) {
    float h = a.hi + a.lo;
    reinterpret_cast<float2 *>(p)[i] = make_float2(h, a.lo - (h - a.hi));
  }
  __device__ static void add_term(DFv &a, float x) { a.add(x); }
  __device__ static double value(const DFv &a) { return a.value(); }
  // a per-arc score sum R[e]: one float (the pair kernels round their
  // compensated sums once when they store them)
  __device__ static void add_arc(DFv &a, const void *R, int64_t i) {
    a.add(reinterpret_cast<const float *>(R)[i]);
  }
};
template <> struct SumT<double> {
  using type = double;
  __device__ static void add_stored(double &a, const void *p, int64_t i) {
    a += reinterpret_cast<const double *>(p)[i];
  }
  __device__ static void store(const double &a, void *p, int64_t i) {
    reinterpret_cast<double *>(p)[i] = a;
  }
  __device__ static void add_term(double &a, double x) { a += x; }
  __device__ static double value(const double &a) { return a; }
  __device__ static void add_arc(double &a, const void *R, int64_t i) {
    a += reinterpret_cast<const double *>(R)[i];
  }
};

// wavefront reductions with a fixed butterfly order
__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
__device__ __forceinline__ double wave_sum_f64(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
__device__ __forceinline__ DFv wave_sum_df(DFv x) {
  for (int off = 32; off > 0; off >>= 1) {
    DFv o;
    o.hi = __shfl_xor(x.hi, off, 64);
    o.lo = __shfl_xor(x.lo, off, 64);
    x.add(o);
  }
  return x;
}
__device__ __forceinline__ DFv wave_sum(DFv x) { return wave_sum_df(x); }
__device__ __forceinline__ void acc_merge(DFv &a, DFv b) { a.add(b); }
__device__ __forceinline__ void acc_merge(double &a, double b) { a += b; }
__device__ __forceinline__ double wave_sum(double x) { return wave_sum_f64(x); }

// Cluster score g(d) = d log d (FP32: log2 units, from v_log_f32) and the
// triangle adjustment delta(sigma) = g(sigma - 6) - g(sigma - 4), taken as the
// difference of two scores: its rounding error is that of scoring the
// triangle cluster itself, the same as every pair term.
__device__ __forceinline__ float score_f(float d) { return d * __builtin_amdgcn_logf(d); }
__device__ __forceinline__ double score_d(double d) { return d * log(d); }

template <typename T> __device__ __forceinline__ T score_t(int32_t d);
template <> __device__ __forceinline__ float score_t<float>(int32_t d) {
  return d > 0 ? score_f((float)d) : 0.0f;
}
template <> __device__ __forceinline__ double score_t<double>(int32_t d) {
  return d > 0 ? score_d((double)d) : 0.0;
}
// g(d) for d >= 0 given as a float/double, without a branch: the log of
// max(d, 1) makes g(0) = 0 (and any negative d, whose result is unused, 0).
__device__ __forceinline__ float score_nn(float d) {
  return d * __builtin_amdgcn_logf(fmaxf(d, 1.0f));
}
__device__ __forceinline__ double score_nn(double d) { return d * log(fmax(d, 1.0)); }

// delta(sigma) = g(sigma - 6) - g(sigma - 4) for the degree sum sigma of a
// triangle's members: each has degree >= 2, so sigma - 4 >= 2 needs no
// guard and g(0) = 0 comes from the log of max(d, 1) (the same values as
// score_t on every sigma >= 6)
template <typename T> __device__ __forceinline__ T tri_delta(int32_t sigma);
template <> __device__ __forceinline__ float tri_delta<float>(int32_t sigma) {
  const float s = (float)sigma, a = s - 6.0f, b = s - 4.0f;
  return a * __builtin_amdgcn_logf(fmaxf(a, 1.0f)) - b * __builtin_amdgcn_logf(b);
}
template <> __device__ __forceinline__ double tri_delta<double>(int32_t sigma) {
  const double s = (double)sigma, a = s - 6.0, b = s - 4.0;
  return a * log(fmax(a, 1.0)) - b * log(b);
}

// ---------------------------------------------------------------------------
// LDS hash set of node ids, open addressing with linear probing (SLOTS a
// power of two; empty = -1). Callers keep at most SLOTS / 2 keys (the tables
// here run at 1/4 or 1/2): a lookup ends at the key or at a free slot, so
// the set must never fill. Hash: multiplicative on the full-rate 24-bit
// multiplier with the high bits folded in first (a 32-bit v_mul_lo runs at a
// quarter of the rate). Slots are single words: a wavefront's random probes
// touch one bank each (4-slot buckets read as 128 bits measured slower).
// ---------------------------------------------------------------------------
template <int SLOTS> struct LdsHash {
  static_assert(SLOTS >= 2 && (SLOTS & (SLOTS - 1)) == 0, "SLOTS must be a power of two");
  static constexpr int kBits = __builtin_ctz(SLOTS);
  __device__ static __forceinline__ uint32_t home(int32_t x) {
    const uint32_t u = (uint32_t)x;
    const uint32_t a = (u ^ (u >> 16)) & 0xFFFFFFu;  // 24-bit operand: v_mul_u32_u24
    return ((a * 0x9E3779u) >> (32 - kBits)) & (uint32_t)(SLOTS - 1);
  }
  // returns the slot taken by x (x not yet in the set)
  __device__ static __forceinline__ int32_t insert(int32_t *keys, int32_t x) {
    uint32_t h = home(x);
    while (atomicCAS(&keys[h], -1, x) != -1) h = (h + 1) & (SLOTS - 1);
    return (int32_t)h;
  }
  // slot of x, or -1
  __device__ static __forceinline__ int32_t find(const int32_t *keys, int32_t x) {
    uint32_t h = home(x);
    int32_t key;
    while ((key = keys[h]) != x && key != -1) h = (h + 1) & (SLOTS - 1);
    return key == x ? (int32_t)h : -1;
  }
};

// ---------------------------------------------------------------------------
// Walking a concatenation of variable-length lists ("segments") with one
// wavefront, 64 consecutive entries per step. segp[s] is the first
// concatenated index of segment s (strictly increasing: no empty segments),
// segp[nseg] = total.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// segment holding entry idx (largest s < nseg with segp[s] <= idx), idx < total
__device__ __forceinline__ int32_t seg_find(const int32_t *segp, int32_t nseg, int32_t idx) {
  int32_t lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (segp[mid] <= idx) lo = mid; else hi = mid;
  }
  return lo;
}

// Per-wavefront LDS scratch of seg_step: 64 flags plus a dummy slot.
constexpr int kFlg = 72;

// One step at entries c .. c+63 with s0 the segment holding entry c (c, s0
// and nseg uniform): returns the segment of this lane's entry c + lane
// (meaningful for c + lane < total) and advances s0 to the segment holding
// entry c + 64. flg is this wavefront's kFlg-word LDS scratch; flags 0..63
// are zero on entry and on return. The starts of segments s0+1 .. s0+64
// inside the step are flagged in LDS and read back as a ballot; p == 64
// marks a start at the next step, lanes past nseg take p = 65 (no segment).
// Branch-free: out-of-step flags land in the dummy slot 64.
__device__ __forceinline__ int32_t seg_step(const int32_t *segp, int32_t nseg, int32_t c,
                                            int32_t &s0, int32_t *flg) {
  const int lane = threadIdx.x & 63;
  wave_sync();  // the previous step's clearing of flg is complete
  const int32_t s = s0 + 1 + lane;
  const int32_t sp = segp[s < nseg ? s : nseg];
  const int32_t p = s <= nseg ? sp - c : 65;
  flg[p < 64 ? p : 64] = 1;
  wave_sync();
  const int32_t f = flg[lane];
  flg[lane] = 0;
  const unsigned long long starts = __ballot(f != 0);
  const int32_t sg = s0 + (int32_t)__builtin_amdgcn_mbcnt_hi(
                              (uint32_t)(starts >> 32),
                              __builtin_amdgcn_mbcnt_lo((uint32_t)starts, 0u)) +
                     (f != 0);
  s0 = __builtin_amdgcn_readfirstlane(s0 + __popcll(starts) +
                                      (int32_t)(__ballot(p == 64) != 0ull));
  return sg;
}

// Walk entries [beg, end) with one wavefront, U steps of 64 per round: the
// segments of all U steps are found first, then every step's load is issued
// (U loads in flight per lane), then the entries are used.
//   load(seg, idx) -> V   reads what entry idx of segment seg needs; lanes
//                         past end call it on entry c of the round (valid)
//   use(seg, idx, V, ok)  consumes it; called on every lane of the wavefront,
//                         ok = (idx < end), V undefined when !ok (so use may
//                         run wavefront-wide operations such as ballots)
//   flush()               after each round (e.g. folds per-round partial sums)
struct NoFlush {
  __device__ void operator()() const {}
};
template <int U, typename Load, typename Use, typename Flush = NoFlush>
__device__ __forceinline__ void seg_walk(const int32_t *segp, int32_t nseg, int32_t beg,
                                         int32_t end, int32_t *flg, Load load, Use use,
                                         Flush flush = Flush()) {
  // uniform bounds in scalar registers: the step conditions become scalar branches
  beg = __builtin_amdgcn_readfirstlane(beg);
  end = __builtin_amdgcn_readfirstlane(end);
  nseg = __builtin_amdgcn_readfirstlane(nseg);
  if (beg >= end) return;
  const int lane = threadIdx.x & 63;
  int32_t s0 = __builtin_amdgcn_readfirstlane(seg_find(segp, nseg, beg));
  for (int32_t c = beg; c < end; c += 64 * U) {
    const int32_t s_c = s0;  // segment of entry c (< end): a valid fallback
    int32_t sg[U];
#pragma unroll
    for (int q = 0; q < U; ++q) sg[q] = (c + 64 * q < end) ? seg_step(segp, nseg, c + 64 * q, s0, flg) : s_c;
    // every lane loads (lanes past end load entry c and ignore it): no
    // branches around the loads, so all U are in flight together
    decltype(load(0, 0)) v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int32_t idx = c + 64 * q + lane;
      const bool ok = idx < end;
      v[q] = load(ok ? sg[q] : s_c, ok ? idx : c);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int32_t idx = c + 64 * q + lane;
      use(sg[q], idx, v[q], idx < end);
    }
    flush();
  }
  wave_sync();
}

// Exclusive scan of one int32 per thread over NT threads (one wavefront, or
// a workgroup of NT/64 wavefronts with `part` = NT/64 ints of LDS); returns
// the exclusive prefix and the group total. Workgroup form: every thread
// must call it (it synchronises twice).
template <int NT>
__device__ __forceinline__ int32_t group_excl_scan(int32_t x, int32_t *part, int32_t &total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t incl = x;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if constexpr (NT == 64) {
    total = __shfl(incl, 63, 64);
    return incl - x;
  } else {
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int w = 0; w < NT / 64; ++w) {
      const int32_t a = part[w];
      if (w < wv) pre += a;
      tot += a;
    }
    __syncthreads();
    total = tot;
    return pre + incl - x;
  }
}

}  // namespace efi
