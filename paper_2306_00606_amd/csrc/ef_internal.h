// Internal declarations shared by the host orchestration (ef_api.cpp) and the
// kernel translation units (*.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ef.h"

namespace efi {

// ---------------------------------------------------------------------------
// Work decomposition constants.
//
// Centres (nodes with k >= 2) are binned by degree k:
//   small  2 <= k <= 64      one wavefront per centre, one 64x64 diagonal tile
//   mid    64 < k <= 1024    one 16-wavefront workgroup per centre
//   big    k > 1024          the pair triangle is cut into super-tiles of
//                            1024 x 1024 neighbours, one workgroup each
// ---------------------------------------------------------------------------
constexpr int kWave = 64;
constexpr int kSmallMax = 64;
constexpr int kSuper = 1024;          // neighbours per super-block
constexpr int kBlocksPerSuper = 16;   // 64-wide blocks per super-block
constexpr int kRecEntries = 2 * kSuper;  // row part + column part per super-tile record

// Triangle pass: a triangle is listed at its middle node w (by rank), with
// an LDS hash of w's degree-oriented out-list up(w). Nodes w with segments
// are binned by |up(w)| and by their walk (tail entries, segments):
//   L: |up| <= kTriLaneM, walk <= kTriLaneWork, segments <= kTriLaneSegs
//      one lane (up(w) and the credits in registers)
//   0: |up| <= kTriBin0, walk <= kTriWaveWork, segments <= kTriWaveSegs
//      one wavefront
//   1: |up| <= kTriBin1     one workgroup (8 wavefronts)
//   2: |up| <= kTriBin2     one workgroup (16 wavefronts)
//   3: longer               binary search of up(w) in global memory
// Largest node degree accepted by the loader: cluster degrees (< 3 * kMaxDegree)
// stay exact in int32, and a degree fits the 20-bit field of the packed
// (degree, position) words of the triangle pass.
constexpr int32_t kMaxDegree = 1000000;
constexpr int kTriBin0 = 64, kTriBin1 = 512, kTriBin2 = 2048;
// Finalize (and surrogate features): nodes of degree <= kFinGroupMax share
// wavefronts, 8 lanes each; degree <= kFinHalfMax: 32 lanes; degree <=
// kFinBlockMin: a wavefront; hubs of degree > kFinBlockMin: a workgroup.
constexpr int32_t kFinGroupMax = 32;
constexpr int32_t kFinLaneMax = 8;  // the cluster finalize: one lane per node up to this degree
constexpr int32_t kFinHalfMax = 512;
constexpr int32_t kFinBlockMin = 4096;
constexpr int kTriLongMin = kTriBin2 + 1;
constexpr int64_t kTriWaveWork = 4096;
constexpr int kTriLaneM = 16;
constexpr int64_t kTriLaneWork = 64;
constexpr int32_t kTriLaneSegs = 64;
static_assert(kTriLaneM < 256 && kTriLaneSegs < 256 && kTriLaneWork < 65536,
              "lane-bin record packing");
constexpr int32_t kTriWaveSegs = 256;
static_assert(kTriBin0 < (1 << 16) && kTriWaveSegs < (1 << 15), "wave-bin record packing");

// Per-seed formulation: seeds are binned by degree k and 2-hop work
// A = sum of neighbour degrees:
//   0: k <= kSeedBin0 and A <= kSeedWaveWork   one wavefront, LDS hash of N(s)
//   1: k <= kSeedBin1                          one workgroup (8 wavefronts)
//   2: k <= kSeedBin2                          one workgroup (16 wavefronts)
//   3: k <= kSeedBin3                          one workgroup, 64 KB LDS hash
//   4: larger                                  one workgroup, bitmap of N(s)
// Hash tables have four times as many slots as keys (twice in bin 3), so a
// miss rarely probes more than a few slots. Neighbour rows are walked in
// chunks of at most kSeedChunk neighbours.
constexpr int kSeedBins = 5;
constexpr int kSeedBin0 = 64, kSeedBin1 = 512, kSeedBin2 = 2048, kSeedBin3 = 8192;
constexpr int64_t kSeedWaveWork = 4096;
constexpr int kSeedChunk = 2048;

// FP32C: seeds whose estimated cancellation factor (S/D)/EF exceeds this are
// recomputed from non-negative terms.
constexpr float kKappaMax = 16.0f;

// Segment-size thresholds of the small bin: a centre of degree k <= 64 is
// scored on segments of 8, 16, 32 or 64 lanes: the first S with k <= t[S]
// (t8 <= 8, t16 <= 16, t32 <= 32; 0 disables a segment size).
// Small centres go to the first bin whose threshold holds their degree:
// bin 0 (k <= t8, at most kSmallLaneMax) one lane per centre; bins 1-3
// (k <= t16, t32, 64) segments of 16, 32, 64 lanes.
constexpr int32_t kSmallLaneMax = 8;
struct SmallThr {
  int32_t t8 = 8, t16 = 16, t32 = 32;
};
__host__ __device__ inline int small_bin(int32_t k, SmallThr t) {
  return k <= t.t8 ? 0 : k <= t.t16 ? 1 : k <= t.t32 ? 2 : 3;
}

struct BigCentre {
  int32_t v;         // node id
  int32_t ns;        // number of super-blocks, ceil(k / 1024)
  int64_t rec_base;  // first super-tile record of this centre
};

struct TileItem {
  int32_t big;  // index into the big-centre list
  int32_t P, Q; // super-block row / column, P <= Q
};

// Device buffer that only grows.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Triangle credits kept with one end of an edge: their sum (64-bit fixed
// point, 2^-36 units: at most 2^20 credits below 2^6 in magnitude each) and
// their count, in one 16-byte record.
struct alignas(16) TriSlot {
  long long y;
  int32_t t;
  int32_t pad;
};
constexpr double kTriFix = 68719476736.0;  // 2^36

// sums over a node's neighbours b of k_b, k_b^2 (exact) and k_b^3, k_b^4
// (FP64: they can pass 2^63)
struct NbrMoments {
  long long s1, s2;
  double s3, s4;
};

struct Graph {
  int dev = 0;
  int32_t n = 0;
  int64_t nnz = 0;
  bool borrowed = false;
  // device arrays
  int32_t *row_ptr = nullptr;
  int32_t *col_idx = nullptr;
  int32_t *deg = nullptr;      // k_v
  int32_t *src = nullptr;      // source node of every arc
  int32_t *rev = nullptr;      // index of the reverse arc
  int32_t *rrev = nullptr;     // where the per-arc sums hold each arc's reverse: rev[e], or,
                               // for an arc into a centre of more than kSmallMax neighbours,
                               // the sorted position (adjs) at which that centre stores its sums
  int2 *adj2 = nullptr;        // (neighbour id, neighbour degree) per arc
  int2 *adjs = nullptr;        // rows of mid and big centres ordered by neighbour degree
                               // (stable): (offset of the arc in its row, neighbour degree);
                               // null when no centre has more than kSmallMax neighbours
  int64_t *asum = nullptr;     // sum of neighbour degrees per node
  longlong2 *qa = nullptr;     // per node: {sum of squared neighbour degrees, sum of neighbours' asum}
  NbrMoments *nbm = nullptr;   // per node: sums of its neighbours' degrees to the powers 1..4,
                               // one 32-byte gather per arc for the surrogate's features
  int32_t *up_ptr = nullptr;   // degree-oriented half adjacency: u -> {w : rank(w) > rank(u)}
  int32_t *up_col = nullptr;   // each up(u) in rank order
  int32_t *up_deg = nullptr;   // degree of every up_col entry
  int32_t *trec = nullptr;     // for every arc v -> a: the triangle record of credits to v, or -1
  // triangle-pass segments of every node w (rows dn_ptr[w] .. dn_ptr[w+1]):
  // {slot of {u, w} in up(u), length of the tail of up(u) above w, k_u, u}
  // for the lower neighbours u of w with a non-empty tail
  int32_t *dn_ptr = nullptr;
  int4 *dn = nullptr;
  // triangle slots (of 2 * up arcs) that no walk writes, cleared on each pass
  int32_t *tri_zero = nullptr;
  int64_t n_tri_zero = 0;
  // host copies used for sizing work lists
  std::vector<int32_t> h_deg;
  std::vector<int32_t> h_up_len;
  // triangle-pass node lists (device): see kTriBin*. Bin 0 as records
  // {w, up_ptr[w], dn_ptr[w], |up(w)| | segments << 16}, bins 1-3 as ids.
  int4 *tri_rec0 = nullptr;
  // lane bin: {w, up_ptr[w], dn_ptr[w], |up(w)| | segments << 8 | walk << 16}, by id
  int4 *tri_recL = nullptr;
  int64_t n_tri_lane = 0;
  int32_t *tri_list[4] = {nullptr, nullptr, nullptr, nullptr};
  // bins 1 and 2 as records too: {w, up_ptr[w], dn_ptr[w], |up(w)| | segments << 12}
  int4 *tri_recB[3] = {nullptr, nullptr, nullptr};
  // nodes of degree > kFinGroupMax (finalized one wavefront each), by degree descending
  int32_t *fin_list = nullptr;
  int64_t n_fin = 0;
  int64_t n_fin_hub = 0;   // leading entries of fin_list with degree > kFinBlockMin
  int64_t n_fin_half = 0;  // trailing entries with degree <= kFinHalfMax
  // after those n_fin entries: the n_fin_group nodes of degree kFinLaneMax+1 ..
  // kFinGroupMax in id order (the cluster finalize takes them 8 lanes each)
  int64_t n_fin_group = 0;
  // per-seed formulation over all nodes: node ids by seed bin (built on first use)
  int32_t *ps_list[kSeedBins] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t n_ps[kSeedBins] = {0, 0, 0, 0, 0};
  bool ps_ready = false;
  std::vector<int64_t> h_asum;  // host copy of asum (built on first per-seed use)
  // graphs loaded as a union of parts (batches): node ids of the triangle
  // lane bin, of triangle bins 0-3 and of fin_list, in list order
  std::vector<int32_t> h_tri_lane, h_tri[4], h_fin;
  std::vector<longlong2> h_qa;  // host copy of qa (built on first three-event use)
  // three-event EF over all nodes: seeds by work, descending, and their item
  // offsets (device, built on first use)
  int32_t *j3_seeds = nullptr;
  int64_t *j3_off = nullptr;
  int64_t n_tri[4] = {0, 0, 0, 0};
  // bin counts for the all-nodes centre set
  int64_t all_small = 0, all_mid = 0, all_big = 0, all_tiles = 0;
  int64_t all_midc[3] = {0, 0, 0};
  int64_t all_small_deg[kSmallMax + 1] = {};  // centres of each degree <= 64
  SmallThr thr;                               // current small-bin thresholds
  // the work lists of a whole-graph call depend only on the graph and thr:
  // built on first use and kept in the work-list buffer (bins_buf) until a
  // call bins other centres, other thresholds, or under stream capture
  bool bins_kept = false;
  SmallThr bins_thr;
  void *bins_buf = nullptr;
  int64_t all_pairs_small = 0, all_pairs_mid = 0, all_pairs_big = 0;
  int64_t all_sblocks = 0;  // sum of super-blocks over big centres
  int64_t owned_bytes = 0;  // device bytes held by this handle
  int32_t *d_counters = nullptr;  // persistent small counters (flag counts etc.)
  ef_graph_info info{};
  ef_run_stats stats{};
  // workspace (grow-only, reused across calls)
  DevBuf ws[16];
  // events for EF_PROFILE
  hipEvent_t ev[16] = {};
  bool ev_ready = false;
};

// ef_compute flag reserved for the library: launch only, no host read-back
// (the call is being captured into a HIP graph)
constexpr uint32_t kInternalNoReadback = 0x80000000u;

// ef_graph_load_csr with the nodes split into n_parts consecutive ranges
// (part_off[n_parts + 1]; null: one part): the node lists are then ordered
// part by part, and their node ids kept on the host
ef_status graph_load(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                     uint32_t flags, void *hip_stream, const int64_t *part_off, int32_t n_parts,
                     ef_graph **out);

// grow-only device scratch held by the graph handle (one slot shared by the
// surrogate entry points)
ef_status graph_scratch(Graph &g, size_t bytes, void **out);

// error text (thread-local)
void set_error(const char *fmt, ...);
ef_status hip_status(hipError_t e, const char *what);

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files). All are asynchronous on `st`
// and return hipSuccess or the launch error.
// ---------------------------------------------------------------------------

// graph preprocessing
int64_t graph_prep_tmp_len(int64_t nnz);
hipError_t launch_graph_prep(Graph &g, int32_t *tmp, int64_t *work, bool &not_symmetric,
                             hipStream_t st);
// Degree-ordered view of the rows of the big centres big[0..nbig) (device
// list): fills g.adjs with a stable segmented sort by neighbour degree.
// scratch: 4 nnz int32 (keys and values, in and out); seg: 2 nbig int32
// (segment ends); temp: the sort's scratch (temp == nullptr: only sets
// temp_bytes).
hipError_t launch_big_sort(Graph &g, const int32_t *big, int32_t nbig, int32_t *scratch,
                           int32_t *seg, void *temp, size_t &temp_bytes, hipStream_t st);
hipError_t graph_zero_count(const Graph &g, const int32_t *tmp, int64_t &count);
hipError_t launch_zero_list(Graph &g, const int32_t *tmp, hipStream_t st);
hipError_t launch_exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t count,
                                     int32_t *block_tmp, int64_t block_tmp_len, hipStream_t st);
int64_t scan_tmp_len(int64_t count);

// flag[0] = 1 if some col[0 .. nnz) lies outside [0, n), else 0 (clears it
// first)
hipError_t launch_check_cols(const int32_t *col, int64_t nnz, int32_t n, int32_t *flag,
                             hipStream_t st);

// zero a small int32 array with a kernel (usable under stream capture)
hipError_t launch_zero_i32(int32_t *p, int32_t count, hipStream_t st);

// work lists
// Mid centres are classed by their number of 64-neighbour blocks: up to 4,
// 5-8, 9-16. The pair kernels give each centre a workgroup of 4, 8 or 16
// wavefronts by class; the persistent batch kernel packs 4, 2 or 1 centres
// into a 16-wavefront workgroup.
__host__ __device__ inline int mid_class(int32_t k) {
  const int nb = (k + 63) >> 6;
  return nb <= 4 ? 0 : nb <= 8 ? 1 : 2;
}

struct Bins {
  SmallThr thr;
  int32_t *small[4] = {nullptr, nullptr, nullptr, nullptr};  // centre ids per segment size
  int64_t n_smallb[4] = {0, 0, 0, 0};
  int32_t *mid = nullptr;
  int32_t *midc[3] = {nullptr, nullptr, nullptr};  // mid centres per class (mid_class)
  int64_t n_midc[3] = {0, 0, 0};
  BigCentre *big = nullptr;
  TileItem *tiles = nullptr;
  int2 *sblocks = nullptr;       // (big-centre index, super-block) reduction items
  int32_t *counters = nullptr;   // [0..3] small, [4] mid, [5] big, [6] tiles, [7] sblocks,
                                 // [8..10] mid classes
  int32_t *agg_done = nullptr;   // per big centre: 1 = pair sums done by aggregation
  int64_t n_small = 0, n_mid = 0, n_big = 0, n_tiles = 0;  // host-known counts
  int64_t pairs_small = 0, pairs_mid = 0, pairs_big = 0;     // clusters per bin
  int64_t n_sblocks = 0;
};
hipError_t launch_bin_centres(const Graph &g, const int32_t *centres, int32_t n_centres,
                              Bins &b, hipStream_t st);

// pair loop: writes R (per arc, base cluster scores without triangle
// correction) for the arcs of every centre in the bins; big centres go via
// super-tile records and a per-arc reduction.
// ev_small / ev_mid / ev_big (nullable) are recorded after the small, mid and
// super-tile kernels.
// agg_done (nullable, one int per big centre): the degree-class aggregated
// variant writes R of big centres directly (1), leaving centres with too many
// distinct neighbour degrees (0) to the super-tile path.
hipError_t launch_pairs(const Graph &g, ef_prec prec, const Bins &b, void *R, void *records,
                        hipStream_t st, hipEvent_t ev_small, hipEvent_t ev_mid,
                        hipEvent_t ev_big, int32_t *agg_done = nullptr);

// triangle pass (cluster-centric): Y, two TriSlots per up arc (upper end at
// the up-arc slot, lower end at nup + slot), Z / ZT per node.
hipError_t launch_triangles(const Graph &g, ef_prec prec, TriSlot *Y, void *Z, int64_t *ZT,
                            hipStream_t st);

// per-node sums + Eq. 1 (cluster-centric); per-node flag bytes in fl.
hipError_t launch_finalize_cluster(const Graph &g, ef_prec prec, const void *R, const TriSlot *Y,
                                   const void *Z, const int64_t *ZT, double *ef, int64_t *D,
                                   int64_t *N, uint8_t *fl, hipStream_t st);

// flag bytes of positions 0..n-1 (written by the finalize and per-seed
// kernels: bit 0 pass 2, bit 1 FP64-finalised) -> flagged list and
// counts[0] (its length), counts[1] (FP64 count); counts are added to.
hipError_t launch_flag_compact(const uint8_t *fl, int64_t n, int32_t *flagged, int32_t *counts,
                               hipStream_t st);

// per-seed formulation: star sums from R of the seed's own arcs, 2-hop walk,
// then Eq. 1. seeds: the unique work list (NULL: position = node id);
// lists[b] / counts[b]: output positions by seed bin (kSeedBins bins, see
// above); the last bin's membership comes from bitmaps, counts[last] of n
// bits each, in list order.
hipError_t launch_per_seed(const Graph &g, ef_prec prec, const int32_t *seeds,
                           const int32_t *const *lists, const int64_t *counts, const void *R,
                           uint32_t *bitmaps, double *ef, int64_t *D, int64_t *N, uint8_t *fl,
                           hipStream_t st, hipEvent_t ev_stream_done);

// Expected Force with three transmission events (j3.hip): items are the arcs
// of seeds[0 .. nseeds), seed i owning items off[i] .. off[i+1]; per-arc
// partial sums in PN / PD / PS. lists: 5 * n_items ints of scratch, counts: 5.
hipError_t launch_j3_items(const Graph &g, bool fp64, const int32_t *seeds, const int64_t *off,
                           int32_t nseeds, int64_t n_items, int32_t *lists, int32_t *counts,
                           long long *PN, long long *PD, double *PS, hipStream_t st);
// N, D, EF of output positions (all of 0 .. count-1, or the count listed in
// pos), node nodes[i] (i when null); FP32C sets fl[i] = 1 where EF cancels.
hipError_t launch_j3_finish(const Graph &g, bool fp64, const long long *PN, const long long *PD,
                            const double *PS, const int32_t *nodes, const int32_t *pos,
                            int32_t count, double *ef, int64_t *D, int64_t *N, uint8_t *fl,
                            hipStream_t st);

// FP32C pass 2: recompute EF of flagged positions from non-negative terms.
// seeds[pos] gives the node of output position pos (NULL: pos is the node).
hipError_t launch_pass2(const Graph &g, const int32_t *seeds, const int32_t *flagged,
                        const int32_t *flag_count, int32_t max_flagged, double *ef,
                        const int64_t *D, hipStream_t st);

// top-k by EF (descending, ties by id ascending) over ef[0..n): device
// values in, device nodes[0..k) and (nullable) ef_out[0..k) out; scratch of
// topk_scratch_bytes(n, k) device bytes, none of it needing prior clearing.
// hipErrorInvalidValue when k > n or the scratch is too small.
size_t topk_scratch_bytes(int32_t n, int32_t k);
hipError_t launch_topk(const double *ef, int32_t n, int32_t k, void *scratch,
                       size_t scratch_bytes, int32_t *nodes, double *ef_out, hipStream_t st);
// the same over non-negative float scores (surrogate predictions)
hipError_t launch_topk_f32(const float *score, int32_t n, int32_t k, void *scratch,
                           size_t scratch_bytes, int32_t *nodes, double *score_out,
                           hipStream_t st);

// Schedule of the persistent batch kernel (one launch for the whole exact
// path of a disjoint union of graphs), all device arrays. Work lists per bin,
// each ordered by graph: pair centres (tiny, 16-, 32-, 64-lane segments, mid
// classes of 4, 2, 1 centres per workgroup), big centres with their
// super-tiles and reduction items, triangle nodes of the wavefront bin
// (records as tri_rec0), of the workgroup bin and of the long bin (ids), and
// finalize nodes of the 8-, 32-, 64-lane and workgroup tiers (the lane tier
// takes node id ranges). items: {type, graph, first, end} into those lists
// (or node ids), in phase order; pend0: items of phases 0, 1, 2 per graph;
// ctl and pend: counters the kernel resets after every launch. The triangle
// lane bin is the graph's own tri_recL.
enum PItemType : int32_t {
  PI_PAIR_LANE = 0, PI_PAIR_S16, PI_PAIR_S32, PI_PAIR_S64, PI_PAIR_M4, PI_PAIR_M2, PI_PAIR_M1,
  PI_PAIR_BIG, PI_TRI_LANE, PI_TRI_WAVE, PI_TRI_BLOCK, PI_TRI_LONG,   // phase 0
  PI_REDUCE,                                                          // phase 1
  PI_FIN_LANE, PI_FIN_G8, PI_FIN_G32, PI_FIN_G64, PI_FIN_HUB,         // phase 2
  PI_PASS2,                                                           // phase 3
  PI_TYPES
};
__host__ __device__ constexpr int pitem_phase(int32_t type) {
  return type <= PI_TRI_LONG ? 0 : type == PI_REDUCE ? 1 : type <= PI_FIN_HUB ? 2 : 3;
}

struct PersistPlan {
  int32_t *pair[7] = {};
  BigCentre *big = nullptr;
  TileItem *tiles = nullptr;
  int2 *reduce = nullptr;
  int4 *tri_wave = nullptr;
  int32_t *tri_block = nullptr, *tri_long = nullptr;
  int32_t *fin_list[4] = {};
  int4 *items = nullptr;
  int32_t n_items = 0, n_graphs = 0;
  int32_t *ctl = nullptr, *pend = nullptr, *pend0 = nullptr;
};
// a persistent-kernel wait longer than this many polls raises the error flag
constexpr int32_t kPersistSpinLimit = 1 << 22;
hipError_t launch_batch_persist(const Graph &g, ef_prec prec, const PersistPlan &pl, void *R,
                                void *rec, TriSlot *Y, void *Z, int64_t *ZT, double *ef,
                                int64_t *D, int64_t *N, uint8_t *fl, hipStream_t st);

// scatter outputs of unique seeds back to the caller's positions
hipError_t launch_gather_outputs(const int32_t *inv, int32_t count, const double *ef_u,
                                 const int64_t *D_u, const int64_t *N_u, double *ef,
                                 int64_t *D, int64_t *N, hipStream_t st);

}  // namespace efi

struct ef_graph {
  efi::Graph g;
};
