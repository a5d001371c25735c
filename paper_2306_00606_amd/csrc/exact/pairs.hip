// Cluster generation and scoring: the pair loop of Algorithm 1.
//
// For a centre v with neighbours a_0 < ... < a_{k-1} (degrees k_p), every
// unordered pair p < q is a cluster (a_p, v, a_q) (Algorithm 1, Phase 1). Its
// degree before the triangle adjustment is d = k_v + k_p + k_q - 4 (Phase 2);
// the triangle adjustment is applied afterwards by the triangle pass. The
// score g(d) = d log d is credited to both ends, so per arc v->a_p we form
//   R[v->a_p] = sum_{q != p} g(k_v + k_p + k_q - 4)
// and every cluster's score is evaluated exactly once.
//
// Layout on a wavefront: lane l holds row p = 64*rb + l of a 64x64 tile and
// keeps the row sum in a register; the column index rotates through the
// wavefront with a DPP wave rotate, together with a rotating column
// accumulator, so after 64 steps each lane holds one column sum. Tiles on the
// diagonal of the pair triangle take 32 steps (each unordered pair once).
//
// Work bins:
//   tiny  (k <= 8)    one lane per centre, its pairs in registers
//   small (k <= 64)   segments of 16, 32 or 64 lanes: one diagonal tile
//   mid   (k <= 1024) one 16-wavefront workgroup per centre: block pairs are
//                     dealt round-robin so every wavefront gets the same load
//   big   (k > 1024)  1024x1024 super-tiles, one workgroup each, written as
//                     records and summed per arc in a fixed order afterwards.
// Column partials cross wavefronts through LDS; every sum has a fixed order,
// so results are bitwise reproducible.
#include <type_traits>

#include "ef_internal.h"

namespace efi {

// the degree of a row or column past the centre's row: -2^21, so that every
// cluster degree d = cp + kq with a masked end stays below 1 (its score is
// +-0) while every value of the degree recurrence, masked or not, is an
// integer of magnitude below 2^24 (exact in FP32)
constexpr float kNegF = -2097152.0f;
constexpr int32_t kNegI = -2097152;  // the same as an integer
static_assert((float)kNegI == kNegF, "kNegI must convert to kNegF");
static_assert(2 * kMaxDegree - 4 + kNegI < 1, "a masked column must give d < 1");
static_assert(3 * kMaxDegree - 2 * kNegI < (1 << 24), "the recurrence must stay exact in FP32");

// ---------------------------------------------------------------------------
// wave rotate: lane l receives the value of lane (l + 1) mod 64
// ---------------------------------------------------------------------------
// bound_ctrl is set: a full rotation has no lane without a source, and with it
// the compiler folds the rotation into the consuming add (v_add_f32_dpp)
__device__ __forceinline__ int rot1i(int x) {
  return __builtin_amdgcn_mov_dpp(x, 0x134, 0xf, 0xf, true);
}
__device__ __forceinline__ float rot1(float x) { return __int_as_float(rot1i(__float_as_int(x))); }
__device__ __forceinline__ double rot1(double x) {
  long long b = __double_as_longlong(x);
  int lo = rot1i((int)(b & 0xffffffffLL));
  int hi = rot1i((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// score of a cluster degree: FP32 path in log2 units (one v_log_f32), FP64
// path in natural-log units.
__device__ __forceinline__ float score(float d) { return d * __builtin_amdgcn_logf(d); }
__device__ __forceinline__ double score(double d) { return d * log(d); }

// score(d) for d >= 1 and +-0 for any d < 1 (masked lanes carry large
// negative degrees), without a branch: integer degrees below 1 give
// log(max(d, 1)) = 0, and adding -0 leaves every sum unchanged
__device__ __forceinline__ float score_masked(float d) {
  return d * __builtin_amdgcn_logf(fmaxf(d, 1.0f));
}
__device__ __forceinline__ double score_masked(double d) { return d * log(fmax(d, 1.0)); }

// ---------------------------------------------------------------------------
// double-float accumulation for the FP32 path
// ---------------------------------------------------------------------------
struct DF {
  float hi, lo;
};
__device__ __forceinline__ void df_add(DF &a, float x) {
  float s = a.hi + x;
  float bb = s - a.hi;
  float e = (a.hi - (s - bb)) + (x - bb);
  a.hi = s;
  a.lo += e;
}
__device__ __forceinline__ DF df_norm(DF a) {
  float h = a.hi + a.lo;
  return DF{h, a.lo - (h - a.hi)};
}

template <typename T> struct Acc;
template <> struct Acc<float> {
  DF v{0.f, 0.f};
  __device__ void add(float x) { df_add(v, x); }
  __device__ void store(void *R, int64_t i) const {
    DF n = df_norm(v);
    reinterpret_cast<float2 *>(R)[i] = make_float2(n.hi, n.lo);
  }
  __device__ void add_stored(const void *R, int64_t i) {
    float2 x = reinterpret_cast<const float2 *>(R)[i];
    df_add(v, x.x);
    df_add(v, x.y);
  }
  // a per-arc sum R[e]: the compensated sum rounded to one float (every term
  // is >= 0, so a node's sum over its arcs keeps a relative error of at most
  // one float rounding from these stores)
  __device__ void store_arc(void *R, int64_t i) const {
    reinterpret_cast<float *>(R)[i] = v.hi + v.lo;
  }
  // a super-tile record entry (a partial over at most 1024 clusters): the
  // compensated sum rounded to one float, half the bytes of a stored pair;
  // the reduction over the records adds the entries compensated again, so a
  // per-arc sum carries one rounding per record entry
  using Rec = float;
  __device__ void store_rec(void *P, int64_t i) const {
    reinterpret_cast<float *>(P)[i] = v.hi + v.lo;
  }
  __device__ static Rec load_rec(const void *P, int64_t i) {
    return reinterpret_cast<const float *>(P)[i];
  }
  __device__ void add_rec(Rec x) { df_add(v, x); }
};
template <> struct Acc<double> {
  double v = 0.0;
  __device__ void add(double x) { v += x; }
  __device__ void store(void *R, int64_t i) const { reinterpret_cast<double *>(R)[i] = v; }
  __device__ void add_stored(const void *R, int64_t i) { v += reinterpret_cast<const double *>(R)[i]; }
  __device__ void store_arc(void *R, int64_t i) const { reinterpret_cast<double *>(R)[i] = v; }
  using Rec = double;
  __device__ void store_rec(void *P, int64_t i) const { reinterpret_cast<double *>(P)[i] = v; }
  __device__ static Rec load_rec(const void *P, int64_t i) {
    return reinterpret_cast<const double *>(P)[i];
  }
  __device__ void add_rec(Rec x) { v += x; }
};

// Full 64x64 tile (no masking) with the row step D = cp - rot(cp) given, so
// that a caller running many tiles of one row block forms it once.
template <typename T>
__device__ __forceinline__ void tile_full(T cp, T kq, T D, T &Rt, T &C) {
  Rt = T(0);
  C = T(0);
  T d = cp + kq;
#pragma unroll 8
  for (int s = 0; s < 64; ++s) {
    T g = score(d);
    Rt += g;
    C = rot1(C) + g;
    d = rot1(d) + D;
  }
}

// ---------------------------------------------------------------------------
// one 64x64 tile on a wavefront
//   cp : k_v + k_p - 4 for this lane's row (kNegF if the row is past k)
//   kq : degree of this lane's column at step 0 (kNegF if past k)
// DIAG: the tile's rows and columns are the same block; steps 1..32, the
//   last step only on lanes 0..31. On return C holds the partial of column
//   (lane + 32) & 63.
// otherwise steps 0..63; on return C holds the partial of column (lane+63)&63.
// MASKED: some rows/columns may be invalid, or d may be 0. Every form steps
//   the cluster degree with the same DPP recurrence; an invalid row or
//   column carries kNegF, which keeps its d below 1 at every step, so its
//   score is zero.
// ---------------------------------------------------------------------------
template <typename T, bool DIAG, bool MASKED>
__device__ __forceinline__ void tile(T cp, T kq, T &Rt, T &C) {
  const int lane = threadIdx.x & 63;
  Rt = T(0);
  C = T(0);
  if (DIAG) {
    // the degree recurrence of the full tiles (below), from step 1
    T d = cp + kq;
    const T D = cp - rot1(cp);
#pragma unroll 4
    for (int s = 1; s <= 32; ++s) {
      d = rot1(d) + D;
      T g = score_masked(d);
      if (s == 32) g = lane < 32 ? g : T(0);
      Rt += g;
      C = rot1(C) + g;
    }
  } else if (MASKED) {
    T d = cp + kq;
    const T D = cp - rot1(cp);
#pragma unroll 8
    for (int s = 0; s < 64; ++s) {
      T g = score_masked(d);
      Rt += g;
      C = rot1(C) + g;
      d = rot1(d) + D;
    }
  } else {
    // d_s(l) = cp(l) + kq(l + s). The lane that holds column q at step s
    // holds column q + 1 at step s + 1, so d_{s+1} = rot(d_s) + cp - rot(cp):
    // one add with the rotation folded in. All values are integers below
    // 2^24, exact in either precision.
    tile_full(cp, kq, cp - rot1(cp), Rt, C);
  }
}

// entries of a big centre's score table (FP32 path)
constexpr int kGTab = 8192;

// Full off-diagonal tile of a big centre with the scores read from the
// centre's table: gt[i] = score(k_v - 2 + i), the same FP32 expression the
// other tiles evaluate, so every cluster gets the same score bits. roff =
// k_p - 2 for this lane's row, kq = degree of its column at step 0; every
// index roff + kq of the tile must lie in the table (checked by the caller).
// Same result layout as tile<T, false, false>; used by the FP32 path.
// The table is addressed by byte offsets idx_s(l) = 4 (roff(l) + kq(l + s)).
// The lane that reads column q at step s reads q + 1 at step s + 1, so
// idx_{s+1} = rot(idx_s) + 4 (roff - rot(roff)): one integer add with the
// rotation folded in (v_add_u32_dpp), as for the cluster degree of tile().
// The difference 4 (roff - rot(roff)) is formed in FP32 (exact: below 2^24):
// folded into an integer v_subrev_u32_dpp it came out negated on the device.
template <typename T>
__device__ __forceinline__ void tile_tab(int32_t roff, int32_t kq, int32_t D, const float *gt,
                                         T &Rt, T &C) {
  Rt = T(0);
  C = T(0);
  const char *base = reinterpret_cast<const char *>(gt);
  int32_t idx = 4 * (roff + kq);
#pragma unroll 8
  for (int s = 0; s < 64; ++s) {
    const T g = *reinterpret_cast<const float *>(base + idx);
    Rt += g;
    C = rot1(C) + g;
    idx = rot1i(idx) + D;
  }
}
// the index step 4 (roff - rot(roff)) of tile_tab for this lane's row
__device__ __forceinline__ int32_t tab_step(int32_t roff) {
  const float r4 = (float)(4 * roff);
  return (int32_t)(r4 - rot1(r4));
}
template <typename T>
__device__ __forceinline__ void tile_tab(int32_t roff, int32_t kq, const float *gt, T &Rt, T &C) {
  tile_tab<T>(roff, kq, tab_step(roff), gt, Rt, C);
}

// ---------------------------------------------------------------------------
// small centres: segments of S lanes (S = 8, 16, 32, 64), one centre of
// degree k <= S per segment, 64/S centres per wavefront. The diagonal tile of
// a segment takes S/2 rotation steps (the last on half of the lanes), so each
// unordered neighbour pair is scored once.
// ---------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ int rot_seg_i(int x) {
  if constexpr (S == 64) {
    return __builtin_amdgcn_mov_dpp(x, 0x134, 0xf, 0xf, true);  // wave_rol:1
  } else if constexpr (S == 16) {
    return __builtin_amdgcn_mov_dpp(x, 0x12F, 0xf, 0xf, true);  // row_ror:15
  } else {
    const int lane = threadIdx.x & 63;
    const int src = (lane & ~(S - 1)) | ((lane + 1) & (S - 1));
    return __builtin_amdgcn_ds_bpermute(src << 2, x);
  }
}
template <int S> __device__ __forceinline__ float rot_seg(float x) {
  return __int_as_float(rot_seg_i<S>(__float_as_int(x)));
}
template <int S> __device__ __forceinline__ double rot_seg(double x) {
  long long b = __double_as_longlong(x);
  int lo = rot_seg_i<S>((int)(b & 0xffffffffLL));
  int hi = rot_seg_i<S>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// one group of 64/S centres (list positions gi*PER ..) on a wavefront
template <typename T, int S>
__device__ __forceinline__ void pairs_seg_group(const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ deg,
                                                const int2 *__restrict__ adj2,
                                                const int32_t *__restrict__ list, int64_t count,
                                                int64_t gi, void *__restrict__ R) {
  constexpr int PER = 64 / S;
  const int lane = threadIdx.x & 63;
  const int seg = lane / S, j = lane & (S - 1);
  const int64_t it = gi * PER + seg;
  const bool have = it < count;
  const int32_t v = have ? list[it] : 0;
  const int32_t k = have ? deg[v] : 0;
  const int32_t base = have ? row_ptr[v] : 0;
  const bool valid = j < k;
  const T kp = valid ? (T)adj2[base + j].y : T(0);
  const T cp = valid ? (T)(k - 4) + kp : (T)kNegF;
  T kq = valid ? kp : (T)kNegF;
  T Rt = T(0), C = T(0);
#pragma unroll 4
  for (int s = 1; s <= S / 2; ++s) {
    kq = rot_seg<S>(kq);
    T g = score_masked(cp + kq);
    if (s == S / 2) g = j < S / 2 ? g : T(0);
    Rt += g;
    C = rot_seg<S>(C) + g;
  }
  // column (j + S/2) mod S is in C of this lane; bring column j home
  const T Cl = __shfl_xor(C, S / 2, 64);
  if (valid) {
    Acc<T> a;
    a.add(Rt);
    a.add(Cl);
    a.store_arc(R, base + j);
  }
}

template <typename T, int S>
__global__ __launch_bounds__(256) void k_pairs_small(const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ deg,
                                                     const int2 *__restrict__ adj2,
                                                     const int32_t *__restrict__ list,
                                                     int64_t count, void *__restrict__ R) {
  constexpr int PER = 64 / S;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t groups = (count + PER - 1) / PER;
  for (int64_t gi = wave; gi < groups; gi += nwaves)
    pairs_seg_group<T, S>(row_ptr, deg, adj2, list, count, gi, R);
}

// ---------------------------------------------------------------------------
// tiny centres (k <= 8): one lane per centre, all C(k, 2) pairs in registers.
// With a few pairs per centre, a segment per centre would spend its time on
// the dependent loads of every centre; a lane keeps 64 centres in flight per
// wavefront. Rows past k are clamped to valid neighbours and masked.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void pairs_lane_one(const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ deg,
                                               const int2 *__restrict__ adj2, int32_t v,
                                               void *__restrict__ R) {
  constexpr int K = kSmallLaneMax;
  const int32_t k = deg[v], base = row_ptr[v];  // 2 <= k <= K
  T kp[K];
#pragma unroll
  for (int p = 0; p < K; ++p) kp[p] = (T)adj2[base + (p < k ? p : k - 1)].y;
  const T c = (T)(k - 4);
  T r[K];
#pragma unroll
  for (int p = 0; p < K; ++p) r[p] = T(0);
#pragma unroll
  for (int p = 0; p < K; ++p) {
#pragma unroll
    for (int q = p + 1; q < K; ++q) {
      const T g = q < k ? score_masked(c + kp[p] + kp[q]) : T(0);
      r[p] += g;
      r[q] += g;
    }
  }
#pragma unroll
  for (int p = 0; p < K; ++p) {
    if (p < k) {
      Acc<T> a;
      a.add(r[p]);
      a.store_arc(R, base + p);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pairs_lane(const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ deg,
                                                    const int2 *__restrict__ adj2,
                                                    const int32_t *__restrict__ list,
                                                    int64_t count, void *__restrict__ R) {
  for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < count;
       it += (int64_t)gridDim.x * blockDim.x)
    pairs_lane_one<T>(row_ptr, deg, adj2, list[it], R);
}

// ---------------------------------------------------------------------------
// shared pieces of the 16-wavefront kernels
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T col_degree(const int2 *adj2, int32_t base, int32_t k, int32_t q) {
  return q < k ? (T)adj2[base + q].y : (T)kNegF;
}

// Diagonal block of blocks (a centre's whole pair triangle for mid centres,
// or a diagonal super-tile for big centres). Blocks blk0 .. blk0+nb-1 of the
// centre's neighbour list; wavefront w (of the group working on this centre)
// owns row block blk0 + w. Every thread of the workgroup calls it the same
// number of times (it holds one workgroup barrier).
// parts[c][delta][64]: column partials, zeroed by the caller; colk: LDS for
// the nb x 64 degrees of the blocks (filled here, behind a barrier).
// On return (after the final barrier), wavefront w's lanes hold in `out` the
// complete sum for index 64*(blk0+w)+lane over all pairs inside this range.
// gtab (FP32, rows in ascending degree order, or null): the centre's score
// table; full off-diagonal tiles whose largest degrees fit read it.
template <typename T>
__device__ void diag_super(const int2 *adj2, int32_t base, int32_t k, T kv4, int blk0, int nb,
                           T (*parts)[9][64], int w, Acc<T> &out, int32_t *colk,
                           const float *gtab = nullptr) {
  const int lane = threadIdx.x & 63;
  const int ws = __builtin_amdgcn_readfirstlane(w);
  const int32_t p = 64 * (blk0 + ws) + lane;
  const bool rvalid = ws < nb && p < k;
  const int32_t kpi = rvalid ? adj2[base + p].y : kNegI;
  // the row degrees of this block of blocks are also its column degrees
  if (ws < nb) colk[64 * ws + lane] = kpi;
  __syncthreads();
  if (ws < nb) {
    const T kp = rvalid ? (T)kpi : T(0);
    const T cp = rvalid ? kv4 + kp : (T)kNegF;
    const int half = nb >> 1;
    const bool ragged = (k & 63) != 0;
    // full column blocks 0 .. nfit-1 fit the table with this row block (the
    // rows of a big centre ascend in degree, so those blocks are a prefix)
    int nfit = 0;
    if (gtab) {
      const int32_t kp_max = __builtin_amdgcn_readlane(kpi, 63);
      bool fit = false;
      if (lane < nb && 64 * (blk0 + lane + 1) <= k) fit = kp_max + colk[64 * lane + 63] - 2 < kGTab;
      nfit = __popcll(__ballot(fit));
    }
    const int32_t Dt = gtab ? tab_step((rvalid ? kpi : 0) - 2) : 0;
    const T Dd = cp - rot1(cp);
    int c = ws;  // column block of round dl: (w + dl) mod nb
    for (int dl = 0; dl <= half; ++dl) {
      if (dl > 0 && dl == half && (nb & 1) == 0 && ws >= half) break;
      T Rt, C;
      if (dl == 0) {
        const T kq = rvalid ? kp : (T)kNegF;
        tile<T, true, true>(cp, kq, Rt, C);
        parts[c][0][(lane + 32) & 63] = C;
      } else {
        const int32_t kq = colk[64 * c + lane];
        const bool masked = ragged && (c == nb - 1 || ws == nb - 1) && (blk0 + nb) * 64 > k;
        if (masked) {
          tile<T, false, true>(cp, (T)kq, Rt, C);
        } else if (c < nfit) {
          tile_tab<T>((rvalid ? kpi : 0) - 2, kq, Dt, gtab, Rt, C);
        } else {
          tile_full<T>(cp, (T)kq, Dd, Rt, C);
        }
        parts[c][dl][(lane + 63) & 63] = C;
      }
      out.add(Rt);
      c = c + 1 == nb ? 0 : c + 1;
    }
  }
  __syncthreads();
  if (ws < nb) {
    const int half = nb >> 1;
    for (int dl = 0; dl <= half; ++dl) out.add(parts[ws][dl][lane]);
  }
}

template <typename T>
__device__ __forceinline__ void zero_parts(T *p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = T(0);
}

// The block pairs of diag_super dealt evenly over the nw wavefronts of a
// group instead of one row block per wavefront: job (dl, r) is row block r
// against column block (r + dl) mod nb, the jobs in dl-major order (the
// dl = 0 jobs are the half-cost diagonal tiles), job j on wavefront j mod nw.
// Row partials go to rowp[r][dl] and column partials to parts[c][dl], one
// writer each; after the barrier wavefront r sums both for its block in a
// fixed order. A centre of 10 blocks on 16 wavefronts takes 3.5 tile times
// instead of 5.5. parts and rowp zeroed by the caller; colk as for
// diag_super. No score table (the rows of mid centres are not in degree
// order).
template <typename T>
__device__ void diag_super_dealt(const int2 *adj2, int32_t base, int32_t k, T kv4, int nb,
                                 T (*parts)[9][64], T (*rowp)[9][64], int w, int nw,
                                 Acc<T> &out, int32_t *colk) {
  const int lane = threadIdx.x & 63;
  const int ws = __builtin_amdgcn_readfirstlane(w);
  if (ws < nb) {
    const int32_t p = 64 * ws + lane;
    colk[64 * ws + lane] = p < k ? adj2[base + p].y : kNegI;
  }
  __syncthreads();
  const int half = nb >> 1;
  const bool ragged = (k & 63) != 0;
  // the even case's last round has only rows 0 .. half-1: the jobs it skips
  // are the last ones of the order
  const int njobs = nb * (half + 1) - ((nb & 1) == 0 ? half : 0);
  for (int j = ws; j < njobs; j += nw) {
    const int dl = j / nb, r = j - dl * nb;
    const int c = r + dl < nb ? r + dl : r + dl - nb;
    const int32_t kpi = colk[64 * r + lane];
    const bool rvalid = 64 * r + lane < k;
    const T kp = rvalid ? (T)kpi : T(0);
    const T cp = rvalid ? kv4 + kp : (T)kNegF;
    T Rt, C;
    if (dl == 0) {
      tile<T, true, true>(cp, rvalid ? kp : (T)kNegF, Rt, C);
      parts[c][0][(lane + 32) & 63] = C;
    } else {
      const T kq = (T)colk[64 * c + lane];
      if (ragged && (c == nb - 1 || r == nb - 1)) tile<T, false, true>(cp, kq, Rt, C);
      else tile_full<T>(cp, kq, cp - rot1(cp), Rt, C);
      parts[c][dl][(lane + 63) & 63] = C;
    }
    rowp[r][dl][lane] = Rt;
  }
  __syncthreads();
  if (ws < nb) {
    for (int dl = 0; dl <= half; ++dl) {
      out.add(rowp[ws][dl][lane]);
      out.add(parts[ws][dl][lane]);
    }
  }
}

// ---------------------------------------------------------------------------
// mid centres (64 < k <= 1024): G centres per workgroup, WPG wavefronts each,
// at least one per block of 64 neighbours. The stand-alone kernels give each
// centre a workgroup of its own (4, 8 or 16 wavefronts for up to 4, 8 or 16
// blocks), so its barriers wait for no other centre and small workgroups
// fill a compute unit eight at a time; the persistent batch kernel packs
// G = 4, 2 or 1 centres into its 16-wavefront workgroups.
// ---------------------------------------------------------------------------
template <typename T, int G, int WPG = kBlocksPerSuper / G> struct MidLdsPlain {
  T parts[G][WPG][9][64];
  int32_t colk[G * WPG * 64];  // each group's degrees, 64 per wavefront
};
// FP32: the block pairs dealt over the group's wavefronts (row partials in
// LDS: 76 KB for 16 wavefronts, two workgroups per CU; 19.5 KB for 4); FP64
// keeps one row block per wavefront (the row partials would take its LDS to
// 148 KB)
template <typename T, int G, int WPG = kBlocksPerSuper / G> struct MidLdsDealt {
  T parts[G][WPG][9][64];
  T rowp[G][WPG][9][64];
  int32_t colk[G * WPG * 64];
};
template <typename T> constexpr bool kMidDealt = std::is_same<T, float>::value;
template <typename T, int G, int WPG = kBlocksPerSuper / G>
using MidLds = typename std::conditional<kMidDealt<T>, MidLdsDealt<T, G, WPG>,
                                         MidLdsPlain<T, G, WPG>>::type;

// centres gi*G .. gi*G+G-1 of the list on a workgroup of G * WPG wavefronts
// (every thread calls it: it holds workgroup barriers); every centre has at
// most WPG blocks of 64 neighbours
template <typename T, int G, int WPG = kBlocksPerSuper / G>
__device__ __forceinline__ void pairs_mid_group(const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ deg,
                                                const int2 *__restrict__ adj2,
                                                const int32_t *__restrict__ list, int64_t count,
                                                int64_t gi, void *__restrict__ R,
                                                MidLds<T, G, WPG> &lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int grp = w / WPG, wl = w % WPG;
  const int64_t it = gi * G + grp;
  const bool have = it < count;  // a group without a centre still meets the barriers
  const int32_t v = have ? list[it] : 0;
  const int32_t k = have ? deg[v] : 0;
  const int32_t base = have ? row_ptr[v] : 0;
  const int nb = (k + 63) >> 6;
  zero_parts(&lds.parts[0][0][0][0], G * WPG * 9 * 64);
  if constexpr (kMidDealt<T>) zero_parts(&lds.rowp[0][0][0][0], G * WPG * 9 * 64);
  __syncthreads();
  Acc<T> out;
  if constexpr (kMidDealt<T>)
    diag_super_dealt<T>(adj2, base, k, (T)(k - 4), nb, lds.parts[grp], lds.rowp[grp], wl, WPG,
                        out, lds.colk + 64 * WPG * grp);
  else
    diag_super<T>(adj2, base, k, (T)(k - 4), 0, nb, lds.parts[grp], wl, out,
                  lds.colk + 64 * WPG * grp);
  const int32_t p = 64 * wl + lane;
  if (wl < nb && p < k) out.store_arc(R, base + p);
  __syncthreads();
}

// one centre per workgroup of WPG wavefronts
template <typename T, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_pairs_mid(const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ deg,
                                                        const int2 *__restrict__ adj2,
                                                        const int32_t *__restrict__ list,
                                                        int64_t count, void *__restrict__ R) {
  __shared__ MidLds<T, 1, WPG> lds;
  for (int64_t gi = blockIdx.x; gi < count; gi += gridDim.x)
    pairs_mid_group<T, 1, WPG>(row_ptr, deg, adj2, list, count, gi, R, lds);
}

// mid centres into their classes (order within a class is not fixed; every
// centre's sums are independent of it)
__global__ __launch_bounds__(256) void k_mid_split(const int32_t *__restrict__ deg,
                                                   const int32_t *__restrict__ mid, int64_t n_mid,
                                                   int32_t *__restrict__ c0,
                                                   int32_t *__restrict__ c1,
                                                   int32_t *__restrict__ c2,
                                                   int32_t *__restrict__ counters) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n_mid;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + lane;
    const int32_t v = i < n_mid ? mid[i] : 0;
    const int c = i < n_mid ? mid_class(deg[v]) : -1;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const unsigned long long m = __ballot(c == q);
      if (m == 0) continue;
      const int lead = __ffsll((unsigned long long)m) - 1;
      int32_t at = 0;
      if (lane == lead) at = atomicAdd(&counters[8 + q], __popcll(m));
      at = __shfl(at, lead, 64);
      int32_t *dst = q == 0 ? c0 : q == 1 ? c1 : c2;
      if (c == q) dst[at + __popcll(m & below)] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// big centres: one workgroup per 1024x1024 super-tile (P, Q), P <= Q, over
// the centre's neighbours in ascending degree (adjs: (offset in the row,
// degree)). record layout, by sorted position:
//                [0, 1024) row part (for P == Q: complete in-range sums),
//                [1024, 2048) column part (P < Q only).
// In the FP32 path a full off-diagonal 64 x 64 tile whose largest row and
// column degrees satisfy k_p + k_q - 2 < kGTab reads its scores from an LDS
// table of score(k_v - 2 + i), i < kGTab, built once per centre and
// workgroup: one LDS read in place of a v_log_f32 and a multiply. In
// degree order that holds for most tiles; the others take the log.
// Column partials of an off-diagonal super-tile: in round dl wavefront w
// takes column block c = (w + dl) mod nbQ, so within a window of kColWin
// rounds the partial of (c, round, w / nbQ) has one writer; a barrier
// between windows orders the adds into the same accumulator, and the
// column sum adds the accumulators in a fixed order (reproducible).
// LDS: table (32 KB), the larger of the diagonal partials (36 KB) and the
// column accumulators (at most 30 KB), and the super-tile's column degrees
// (4 KB), so that two workgroups fit on a compute unit.
// ---------------------------------------------------------------------------
constexpr int kColWin = 4;  // rounds between the barriers of the column adds

// most (column block, wavefront group) pairs of one round over nbQ <= 16
// blocks: nbQ * ceil(16 / nbQ), largest at nbQ = 15
__host__ __device__ constexpr int col_groups_max() {
  int m = 0;
  for (int nb = 1; nb <= kBlocksPerSuper; ++nb) {
    const int g = nb * ((kBlocksPerSuper + nb - 1) / nb);
    m = g > m ? g : m;
  }
  return m;
}

template <typename T> struct BigLds {
  static constexpr bool kTab = std::is_same<T, float>::value;
  static constexpr int kTabBytes = kTab ? kGTab * 4 : 0;
  static constexpr int kDiagBytes = kBlocksPerSuper * 9 * 64 * (int)sizeof(T);
  static constexpr int kColBytes = col_groups_max() * kColWin * 64 * (int)sizeof(T);
  static constexpr int kPartBytes = kDiagBytes > kColBytes ? kDiagBytes : kColBytes;
  static constexpr int kColDegBytes = kSuper * 4;  // column degrees of the super-tile
  static constexpr int kBytes = kTabBytes + kPartBytes + kColDegBytes;
};


// One super-tile on a 16-wavefront workgroup (every thread calls it: it holds
// workgroup barriers). lds: BigLds<T>::kBytes, the scores of the current
// centre (FP32 path) first, at address 0, so that a table read needs no base
// added; then the partials. tab_v: the centre whose scores lds holds (-1:
// none), kept by the caller across calls.
template <typename T>
__device__ __forceinline__ void pairs_big_tile(const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ deg,
                                               const int2 *__restrict__ adjs,
                                               const BigCentre *__restrict__ big,
                                               const TileItem ti, void *__restrict__ rec,
                                               unsigned char *lds, int32_t &tab_v) {
  constexpr bool kTab = BigLds<T>::kTab;
  float *gtab = reinterpret_cast<float *>(lds);
  T(*parts)[9][64] = reinterpret_cast<T(*)[9][64]>(lds + BigLds<T>::kTabBytes);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int2 *adj2 = adjs;
  const BigCentre bc = big[ti.big];
  const int32_t v = bc.v, k = deg[v], base = row_ptr[v], ns = bc.ns;
  const int P = ti.P, Q = ti.Q;
  const int64_t tile_idx = bc.rec_base + (int64_t)P * ns - (int64_t)P * (P - 1) / 2 + (Q - P);
  const int64_t rbase = tile_idx * kRecEntries;
  const int nbQ = min(kBlocksPerSuper, (k - kSuper * Q + 63) >> 6);
  const T kv4 = (T)(k - 4);
  if (P == Q) {
    if (kTab && v != tab_v) {  // uniform: one centre per work item
      const float d0 = (float)(k - 2);
      for (int i = threadIdx.x; i < kGTab; i += blockDim.x) gtab[i] = score(d0 + (float)i);
      tab_v = v;
    }
    zero_parts(&parts[0][0][0], kBlocksPerSuper * 9 * 64);
    __syncthreads();
    Acc<T> out;
    // the rows of a big centre ascend in degree, so its full off-diagonal
    // tiles can read the score table here too
    diag_super<T>(adj2, base, k, kv4, kBlocksPerSuper * P, nbQ,
                  reinterpret_cast<T(*)[9][64]>(&parts[0][0][0]), w, out,
                  reinterpret_cast<int32_t *>(lds + BigLds<T>::kTabBytes + BigLds<T>::kPartBytes),
                  kTab ? gtab : nullptr);
    if (w < nbQ) out.store_rec(rec, rbase + 64 * w + lane);
  } else {
    // P < Q: all 16 row blocks of P are full
    const int ws = __builtin_amdgcn_readfirstlane(w);
    const int32_t p = kSuper * P + 64 * w + lane;
    const int32_t kp = adj2[base + p].y;
    const T cp = kv4 + (T)kp;
    const bool ragged_q = (kSuper * Q + 64 * nbQ) > k;
    // G wavefronts share a column block in one round (G = 1 when nbQ = 16)
    const int G = (kBlocksPerSuper + nbQ - 1) / nbQ;
    T *cacc = &parts[0][0][0];
    int32_t *colk = reinterpret_cast<int32_t *>(lds + BigLds<T>::kTabBytes + BigLds<T>::kPartBytes);
    zero_parts(cacc, nbQ * G * kColWin * 64);
    for (int i = threadIdx.x; i < 64 * nbQ; i += blockDim.x) {
      const int32_t q = kSuper * Q + i;
      colk[i] = q < k ? adj2[base + q].y : kNegI;
    }
    if (kTab && v != tab_v) {  // uniform: one centre per work item
      const float d0 = (float)(k - 2);
      for (int i = threadIdx.x; i < kGTab; i += blockDim.x) gtab[i] = score(d0 + (float)i);
      tab_v = v;
    }
    __syncthreads();
    // full column blocks 0 .. nfit-1 fit the table for this wavefront's rows:
    // k_p + k_q - 2 < kGTab at the largest row and column degrees (the last
    // lane of each block, as degrees ascend, so the blocks that fit are a
    // prefix)
    int nfit = 0;
    if (kTab) {
      const int32_t kp_max = __shfl(kp, 63, 64);
      const int nfull = ragged_q ? nbQ - 1 : nbQ;
      bool fit = false;
      if (lane < nfull) fit = kp_max + colk[64 * lane + 63] - 2 < kGTab;
      nfit = __popcll(__ballot(fit));
    }
    const int32_t Dt = kTab ? tab_step(kp - 2) : 0;
    const T Dd = cp - rot1(cp);
    Acc<T> out;
    T *mine = cacc + ((w / nbQ) * kColWin) * 64 + ((lane + 63) & 63);
    int c = ws % nbQ;  // column block of round dl: (w + dl) mod nbQ
    for (int dl = 0; dl < nbQ; ++dl) {
      const int32_t kq = colk[64 * c + lane];
      T Rt, C;
      if (ragged_q && c == nbQ - 1) {
        tile<T, false, true>(cp, (T)kq, Rt, C);
      } else if (c < nfit) {
        tile_tab<T>(kp - 2, kq, Dt, gtab, Rt, C);
      } else {
        tile_full<T>(cp, (T)kq, Dd, Rt, C);
      }
      // accumulator (c, w / nbQ, dl mod kColWin): one writer in this window
      mine[(c * G * kColWin + dl % kColWin) * 64] += C;
      out.add(Rt);
      if (dl % kColWin == kColWin - 1 && dl + 1 < nbQ) __syncthreads();
      c = c + 1 == nbQ ? 0 : c + 1;
    }
    out.store_rec(rec, rbase + 64 * w + lane);
    __syncthreads();
    {
      const int cc = threadIdx.x >> 6, j = threadIdx.x & 63;
      if (cc < nbQ) {
        Acc<T> col;
        const T *a = cacc + cc * G * kColWin * 64 + j;
        for (int i = 0; i < G * kColWin; ++i) col.add(a[64 * i]);
        col.store_rec(rec, rbase + kSuper + 64 * cc + j);
      }
    }
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(1024) void k_pairs_big(const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ deg,
                                                    const int2 *__restrict__ adjs,
                                                    const BigCentre *__restrict__ big,
                                                    const TileItem *__restrict__ tiles,
                                                    int64_t count, void *__restrict__ rec,
                                                    const int32_t *__restrict__ agg_done) {
  __shared__ __align__(16) unsigned char lds[BigLds<T>::kBytes];
  int32_t tab_v = -1;  // centre whose scores the table holds
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const TileItem ti = tiles[it];
    if (agg_done && agg_done[ti.big]) continue;  // uniform per workgroup
    pairs_big_tile<T>(row_ptr, deg, adjs, big, ti, rec, lds, tab_v);
  }
}

// ---------------------------------------------------------------------------
// Degree-class aggregation of the pair loop for big centres (a variant of
// Algorithm 1, Phase 2 that reaches the same per-arc sums): with c = k_v - 4
// and m_j neighbours of degree kappa_j,
//   R[v->a_p] = sum_{q != p} g(c + k_p + k_q)
//             = T(k_p) - g(c + 2 k_p),   T(kappa) = sum_j m_j g(c + kappa + kappa_j),
// so a centre costs M^2 score evaluations (M distinct neighbour degrees)
// instead of k(k-1)/2. One workgroup per big centre:
//   1. histogram of neighbour degrees in an LDS hash (kAggSlots slots, at
//      most kAggMax distinct; beyond that the centre is left to the
//      super-tile path: agg_done[bi] = 0);
//   2. distinct degrees sorted ascending (bitonic sort in LDS), so every sum
//      has a fixed order and results are reproducible;
//   3. T for every distinct degree (row i: sum over j ascending);
//   4. R for every arc from T.
// ---------------------------------------------------------------------------
constexpr int kAggMax = 4096;    // distinct neighbour degrees per centre
constexpr int kAggSlots = 8192;  // hash slots (load factor <= 1/2)

template <typename T>
__global__ __launch_bounds__(1024) void k_pairs_agg(const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ deg,
                                                    const int2 *__restrict__ adjs,
                                                    const BigCentre *__restrict__ big,
                                                    const int32_t *__restrict__ counters,
                                                    int32_t *__restrict__ agg_done,
                                                    void *__restrict__ R) {
  __shared__ int32_t hkey[kAggSlots];
  __shared__ int32_t hval[kAggSlots];  // count, then the sorted index
  __shared__ int32_t skey[kAggMax];
  __shared__ int32_t scnt[kAggMax];
  __shared__ T tsum[(sizeof(T) == 4 ? 2 : 1) * kAggMax];  // FP32: (hi, lo) pairs; FP64: one value
  __shared__ int32_t nd_s, over_s;
  constexpr uint32_t kMask = kAggSlots - 1;
  const int tid = threadIdx.x;
  const int32_t nbig = counters[5];
  for (int32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const BigCentre bc = big[bi];
    const int32_t v = bc.v, k = deg[v], base = row_ptr[v];
    const T c = (T)(k - 4);
    for (int i = tid; i < kAggSlots; i += 1024) {
      hkey[i] = -1;
      hval[i] = 0;
    }
    if (tid == 0) {
      nd_s = 0;
      over_s = 0;
    }
    __syncthreads();
    // 1. histogram (find-or-insert; a probe gives up after kAggSlots slots)
    for (int32_t e = base + tid; e < base + k; e += 1024) {
      const int32_t kap = adjs[e].y;
      uint32_t h = ((uint32_t)kap * 0x9E3779u) & kMask;
      for (int t = 0; t < kAggSlots; ++t) {
        const int32_t cur = atomicCAS(&hkey[h], -1, kap);
        if (cur == -1) {
          if (atomicAdd(&nd_s, 1) >= kAggMax) over_s = 1;
        }
        if (cur == -1 || cur == kap) {
          atomicAdd(&hval[h], 1);
          break;
        }
        h = (h + 1) & kMask;
      }
    }
    __syncthreads();
    if (over_s) {
      if (tid == 0) agg_done[bi] = 0;
      __syncthreads();
      continue;
    }
    const int32_t M = nd_s;
    int32_t P = 1;
    while (P < M) P <<= 1;
    // 2. compact (any order), pad to P with +inf keys, bitonic sort ascending
    for (int i = tid; i < P; i += 1024) {
      skey[i] = 0x7fffffff;
      scnt[i] = 0;
    }
    __syncthreads();
    if (tid == 0) nd_s = 0;
    __syncthreads();
    for (int i = tid; i < kAggSlots; i += 1024) {
      if (hkey[i] >= 0) {
        const int32_t pos = atomicAdd(&nd_s, 1);
        skey[pos] = hkey[i];
        scnt[pos] = hval[i];
      }
    }
    __syncthreads();
    for (int len = 2; len <= P; len <<= 1) {
      for (int stride = len >> 1; stride > 0; stride >>= 1) {
        for (int i = tid; i < P; i += 1024) {
          const int j = i ^ stride;
          if (j > i) {
            const bool up = (i & len) == 0;
            const int32_t a = skey[i], b2 = skey[j];
            if ((a > b2) == up) {
              skey[i] = b2;
              skey[j] = a;
              const int32_t t2 = scnt[i];
              scnt[i] = scnt[j];
              scnt[j] = t2;
            }
          }
        }
        __syncthreads();
      }
    }
    // sorted index of each distinct degree, kept in the hash value slot
    for (int i = tid; i < M; i += 1024) {
      const int32_t kap = skey[i];
      uint32_t h = ((uint32_t)kap * 0x9E3779u) & kMask;
      while (hkey[h] != kap) h = (h + 1) & kMask;
      hval[h] = i;
    }
    // 3. T(kappa_i) = sum_j m_j g(c + kappa_i + kappa_j), j ascending
    for (int i = tid; i < M; i += 1024) {
      const T ci = c + (T)skey[i];
      Acc<T> a;
      for (int j = 0; j < M; ++j) a.add((T)scnt[j] * score(ci + (T)skey[j]));
      a.store(tsum, i);
    }
    __syncthreads();
    // 4. R = T(k_p) - g(c + 2 k_p), stored by sorted position like the
    // super-tile sums of a big centre
    for (int32_t e = base + tid; e < base + k; e += 1024) {
      const int32_t kap = adjs[e].y;
      uint32_t h = ((uint32_t)kap * 0x9E3779u) & kMask;
      while (hkey[h] != kap) h = (h + 1) & kMask;
      Acc<T> a;
      a.add_stored(tsum, hval[h]);
      a.add(-score(c + (T)(2 * kap)));
      a.store_arc(R, e);
    }
    if (tid == 0) agg_done[bi] = 1;
    __syncthreads();
  }
}

// Per-arc sum of the super-tile records of big centres, fixed order, for the
// neighbour at sorted position p (stored at base + p: a big centre keeps its
// row's sums in sorted order; Graph::rrev points each reverse arc there):
// R = sum_{Q >= b} row part of (b, Q)  +  sum_{P < b} column part of (P, b)
// One workgroup per (big centre, super-block b): the 1024 arcs of block b.
template <typename T>
__device__ __forceinline__ void arc_reduce_item(const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ deg,
                                                const int2 *__restrict__ adjs,
                                                const BigCentre *__restrict__ big,
                                                const int2 item, const void *__restrict__ rec,
                                                void *__restrict__ R) {
  const BigCentre bc = big[item.x];
  const int b = item.y;
  const int32_t k = deg[bc.v], base = row_ptr[bc.v], ns = bc.ns;
  // entry j of the row part of (b, Q) and of the column part of (P, b)
  const int64_t row0 = (bc.rec_base + (int64_t)b * ns - (int64_t)b * (b - 1) / 2 - b) * kRecEntries;
  auto rowi = [&](int Q, int j) { return row0 + (int64_t)Q * kRecEntries + j; };
  auto coli = [&](int P, int j) {
    return (bc.rec_base + (int64_t)P * ns - (int64_t)P * (P - 1) / 2 + (b - P)) * kRecEntries +
           kSuper + j;
  };
  using Rec = typename Acc<T>::Rec;
  for (int j = threadIdx.x; j < kSuper; j += blockDim.x) {
    const int32_t p = kSuper * b + j;
    if (p >= k) break;
    Acc<T> a;
    // four reads in flight, added in the same order
    int Q = b;
    for (; Q + 3 < ns; Q += 4) {
      const Rec r0 = Acc<T>::load_rec(rec, rowi(Q, j)), r1 = Acc<T>::load_rec(rec, rowi(Q + 1, j)),
                r2 = Acc<T>::load_rec(rec, rowi(Q + 2, j)),
                r3 = Acc<T>::load_rec(rec, rowi(Q + 3, j));
      a.add_rec(r0);
      a.add_rec(r1);
      a.add_rec(r2);
      a.add_rec(r3);
    }
    for (; Q < ns; ++Q) a.add_rec(Acc<T>::load_rec(rec, rowi(Q, j)));
    int P = 0;
    for (; P + 3 < b; P += 4) {
      const Rec r0 = Acc<T>::load_rec(rec, coli(P, j)), r1 = Acc<T>::load_rec(rec, coli(P + 1, j)),
                r2 = Acc<T>::load_rec(rec, coli(P + 2, j)),
                r3 = Acc<T>::load_rec(rec, coli(P + 3, j));
      a.add_rec(r0);
      a.add_rec(r1);
      a.add_rec(r2);
      a.add_rec(r3);
    }
    for (; P < b; ++P) a.add_rec(Acc<T>::load_rec(rec, coli(P, j)));
    a.store_arc(R, base + p);  // by sorted position (a big centre's row layout)
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_arc_reduce(const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ deg,
                                                    const int2 *__restrict__ adjs,
                                                    const BigCentre *__restrict__ big,
                                                    const int2 *__restrict__ items,
                                                    int64_t nitems, const void *__restrict__ rec,
                                                    void *__restrict__ R,
                                                    const int32_t *__restrict__ agg_done) {
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    if (agg_done && agg_done[item.x]) continue;
    arc_reduce_item<T>(row_ptr, deg, adjs, big, item, rec, R);
  }
}

// ---------------------------------------------------------------------------
// binning: classify centres by degree and build the work lists.
// counters: [0..3] small lists (segments of 8, 16, 32, 64 lanes), [4] mid,
// [5] big, [6] super-tile records, [7] super-block reduction items.
// A small centre of degree k goes to the first segment size S with
// k <= thr[S] (thr[64] = 64), so the thresholds pick the segment size.
// ---------------------------------------------------------------------------
// binning: each workgroup classifies 256 * kBinPer centres per round; ranks
// within a bin come from wavefront ballots (and, for the big bin, a scan of
// super-tile counts), per-wavefront counts meet in LDS, and each bin takes one
// global atomic per workgroup and round: device-scope atomics on one address
// serialise across the XCDs.
constexpr int kBinPer = 8;

__global__ __launch_bounds__(256) void k_bin(const int32_t *__restrict__ deg,
                                             const int32_t *__restrict__ centres,
                                             int32_t n_centres, SmallThr thr,
                                             int32_t *__restrict__ small0,
                                             int32_t *__restrict__ small1,
                                             int32_t *__restrict__ small2,
                                             int32_t *__restrict__ small3,
                                             int32_t *__restrict__ mid,
                                             BigCentre *__restrict__ big,
                                             int32_t *__restrict__ counters) {
  // bins 0..3 small, 4 mid, 5 big (centres), 6 big (super-tiles)
  __shared__ int32_t wcnt[4][7];
  __shared__ int32_t gbase[7];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  constexpr int64_t kRound = 256 * kBinPer;
  for (int64_t r0 = blockIdx.x * kRound; r0 < n_centres; r0 += (int64_t)gridDim.x * kRound) {
    int32_t vv[kBinPer], rank[kBinPer], tpre[kBinPer], nsb[kBinPer];
    int bb[kBinPer];
    int32_t run[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < kBinPer; ++j) {
      const int64_t i = r0 + (int64_t)(j * 4 + wv) * 64 + lane;
      int32_t v = 0, k = 0;
      if (i < n_centres) {
        v = centres ? centres[i] : (int32_t)i;
        k = deg[v];
      }
      const int b = (k < 2) ? -1 : k <= kSmallMax ? small_bin(k, thr) : k <= kSuper ? 4 : 5;
      vv[j] = v;
      bb[j] = b;
      rank[j] = 0;
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const unsigned long long m = __ballot(b == q);
        if (b == q) rank[j] = run[q] + __popcll(m & below);
        run[q] += __popcll(m);
      }
      // super-tiles of big centres: exclusive scan within the wavefront
      const int32_t ns = b == 5 ? (k + kSuper - 1) / kSuper : 0;
      const int32_t nt = ns * (ns + 1) / 2;
      int32_t incl = nt;
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
      }
      nsb[j] = ns;
      tpre[j] = run[6] + incl - nt;
      run[6] += __shfl(incl, 63, 64);
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 7; ++q) wcnt[wv][q] = run[q];
    }
    __syncthreads();
    if (tid < 7) {
      const int32_t tot = wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
      gbase[tid] = tot ? atomicAdd(&counters[tid], tot) : 0;
    }
    __syncthreads();
    int32_t off[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      int32_t o = gbase[q];
      for (int w = 0; w < wv; ++w) o += wcnt[w][q];
      off[q] = o;
    }
#pragma unroll
    for (int j = 0; j < kBinPer; ++j) {
      const int b = bb[j];
      if (b < 0) continue;
      if (b == 5) {
        big[off[5] + rank[j]] = BigCentre{vv[j], nsb[j], (int64_t)(off[6] + tpre[j])};
        continue;
      }
      const int32_t pos = (b == 0 ? off[0] : b == 1 ? off[1] : b == 2 ? off[2] : b == 3 ? off[3]
                                                                                      : off[4]) +
                          rank[j];
      int32_t *list = b == 0 ? small0 : b == 1 ? small1 : b == 2 ? small2 : b == 3 ? small3 : mid;
      list[pos] = vv[j];
    }
    __syncthreads();
  }
}

// one workgroup per big centre: its super-tile items (in record order)
__global__ void k_expand_tiles(const BigCentre *__restrict__ big, int32_t *__restrict__ counters,
                               TileItem *__restrict__ tiles, int2 *__restrict__ sblocks) {
  const int32_t nbig = counters[5];
  for (int32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const BigCentre bc = big[bi];
    const int32_t nt = bc.ns * (bc.ns + 1) / 2;
    __shared__ int32_t sb0;
    if (threadIdx.x == 0) sb0 = atomicAdd(&counters[7], bc.ns);
    __syncthreads();
    for (int32_t b = threadIdx.x; b < bc.ns; b += blockDim.x) sblocks[sb0 + b] = make_int2(bi, b);
    __syncthreads();
    for (int32_t t = threadIdx.x; t < nt; t += blockDim.x) {
      // invert t = P*ns - P*(P-1)/2 + (Q-P)
      int32_t P = 0, rem = t;
      while (rem >= bc.ns - P) { rem -= bc.ns - P; ++P; }
      tiles[bc.rec_base + t] = TileItem{bi, P, P + rem};
    }
  }
}

__global__ void k_zero_i32(int32_t *__restrict__ p, int32_t count) {
  for (int32_t i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

hipError_t launch_zero_i32(int32_t *p, int32_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, st, p, count);
  return hipGetLastError();
}

static unsigned capped(int64_t blocks, int64_t cap) {
  if (blocks < 1) blocks = 1;
  return (unsigned)(blocks < cap ? blocks : cap);
}

hipError_t launch_bin_centres(const Graph &g, const int32_t *centres, int32_t n_centres,
                              Bins &b, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, b.counters, 16);
  if (n_centres <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin, dim3(capped((n_centres + 256 * kBinPer - 1) / (256 * kBinPer), 4096)),
                     dim3(256), 0, st,
                     g.deg, centres, n_centres, b.thr, b.small[0], b.small[1], b.small[2],
                     b.small[3], b.mid, b.big, b.counters);
  if (b.n_big > 0)
    hipLaunchKernelGGL(k_expand_tiles, dim3(capped(b.n_big, 65536)), dim3(256), 0, st, b.big,
                       b.counters, b.tiles, b.sblocks);
  if (b.n_mid > 0)
    hipLaunchKernelGGL(k_mid_split, dim3(capped((b.n_mid + 255) / 256, 4096)), dim3(256), 0, st,
                       g.deg, b.mid, b.n_mid, b.midc[0], b.midc[1], b.midc[2], b.counters);
  return hipGetLastError();
}

template <typename T>
static hipError_t pairs_impl(const Graph &g, const Bins &b, void *R, void *records,
                             hipStream_t st, hipEvent_t ev_small, hipEvent_t ev_mid,
                             hipEvent_t ev_big, int32_t *agg_done) {
  static_assert(kSmallLaneMax == 8, "bin 0 holds centres of degree <= 8, one lane each");
  if (b.n_smallb[0] > 0)
    hipLaunchKernelGGL(k_pairs_lane<T>, dim3(capped((b.n_smallb[0] + 255) / 256, 1 << 16)),
                       dim3(256), 0, st, g.row_ptr, g.deg, g.adj2, b.small[0], b.n_smallb[0], R);
  if (b.n_smallb[1] > 0)
    hipLaunchKernelGGL((k_pairs_small<T, 16>), dim3(capped((b.n_smallb[1] + 15) / 16, 1 << 20)),
                       dim3(256), 0, st, g.row_ptr, g.deg, g.adj2, b.small[1], b.n_smallb[1], R);
  if (b.n_smallb[2] > 0)
    hipLaunchKernelGGL((k_pairs_small<T, 32>), dim3(capped((b.n_smallb[2] + 7) / 8, 1 << 20)),
                       dim3(256), 0, st, g.row_ptr, g.deg, g.adj2, b.small[2], b.n_smallb[2], R);
  if (b.n_smallb[3] > 0)
    hipLaunchKernelGGL((k_pairs_small<T, 64>), dim3(capped((b.n_smallb[3] + 3) / 4, 1 << 20)),
                       dim3(256), 0, st, g.row_ptr, g.deg, g.adj2, b.small[3], b.n_smallb[3], R);
  if (ev_small) (void)hipEventRecord(ev_small, st);
  // class c holds centres of up to 4 << c blocks: one workgroup of that
  // many wavefronts each, over the degree-ordered rows (adjs), so that the
  // per-arc sums go out by sorted position like a big centre's
  if (b.n_midc[0] > 0)
    hipLaunchKernelGGL((k_pairs_mid<T, 4>), dim3(capped(b.n_midc[0], 1 << 20)), dim3(256), 0,
                       st, g.row_ptr, g.deg, g.adjs, b.midc[0], b.n_midc[0], R);
  if (b.n_midc[1] > 0)
    hipLaunchKernelGGL((k_pairs_mid<T, 8>), dim3(capped(b.n_midc[1], 1 << 20)), dim3(512), 0,
                       st, g.row_ptr, g.deg, g.adjs, b.midc[1], b.n_midc[1], R);
  if (b.n_midc[2] > 0)
    hipLaunchKernelGGL((k_pairs_mid<T, 16>), dim3(capped(b.n_midc[2], 1 << 20)), dim3(1024), 0,
                       st, g.row_ptr, g.deg, g.adjs, b.midc[2], b.n_midc[2], R);
  if (ev_mid) (void)hipEventRecord(ev_mid, st);
  if (agg_done && b.n_big > 0)
    hipLaunchKernelGGL(k_pairs_agg<T>, dim3(capped(b.n_big, 1 << 16)), dim3(1024), 0, st,
                       g.row_ptr, g.deg, g.adjs, b.big, b.counters, agg_done, R);
  if (b.n_tiles > 0)
    hipLaunchKernelGGL(k_pairs_big<T>, dim3(capped(b.n_tiles, 1 << 20)), dim3(1024), 0, st,
                       g.row_ptr, g.deg, g.adjs, b.big, b.tiles, b.n_tiles, records, agg_done);
  if (ev_big) (void)hipEventRecord(ev_big, st);
  if (b.n_sblocks > 0)
    hipLaunchKernelGGL(k_arc_reduce<T>, dim3(capped(b.n_sblocks, 1 << 20)), dim3(256), 0, st,
                       g.row_ptr, g.deg, g.adjs, b.big, b.sblocks, b.n_sblocks, records, R,
                       agg_done);
  return hipGetLastError();
}

hipError_t launch_pairs(const Graph &g, ef_prec prec, const Bins &b, void *R, void *records,
                        hipStream_t st, hipEvent_t ev_small, hipEvent_t ev_mid,
                        hipEvent_t ev_big, int32_t *agg_done) {
  if (prec == EF_PREC_FP64)
    return pairs_impl<double>(g, b, R, records, st, ev_small, ev_mid, ev_big, agg_done);
  return pairs_impl<float>(g, b, R, records, st, ev_small, ev_mid, ev_big, agg_done);
}

}  // namespace efi
