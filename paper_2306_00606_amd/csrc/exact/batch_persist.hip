// Persistent batch kernel: the whole exact path of a batch of graphs (pair
// loop, triangle pass, per-node sums and Eq. 1, FP32 pass 2) from a single
// launch.
//
// The batch is a disjoint union, and a cluster never spans two graphs
// (Sec. 3.3), so the work of one graph depends only on that graph. Work items
// (a chunk of one bin of one graph) sit in one list, in phase order:
//   phase 0  pair loop and triangle pass (independent of each other)
//   phase 1  per-arc sums of big centres' super-tile records
//   phase 2  per-node sums and Eq. 1
//   phase 3  pass 2 of the seeds whose EF cancels
// A grid of resident workgroups takes items from an atomic cursor. An item of
// phase p waits until its graph has no item of an earlier phase left
// (per-graph counters). Every such item was taken from the cursor before this
// one, by a workgroup that is running it and waits only for still earlier
// phases, so the waits end without any assumption on how many workgroups are
// resident. Each wait is bounded all the same: past the limit the item is
// dropped and an error flag is raised instead of spinning on.
//
// Producers make their stores visible at device scope before they count an
// item done (release fence in every wavefront, then one atomic); consumers
// acquire after the wait. The last workgroup to leave resets the cursor and
// counters for the next launch, so one launch is the whole pass and the
// launch can be captured and replayed.
//
// The item bodies are the device functions of the separate kernels (the
// same code), run by 16-wavefront workgroups with one LDS pool shared by all
// item types.

namespace efi {

// triangle bins of the persistent kernel: wavefront nodes with their own
// LDS state (|up(w)| <= 64 at load factor 1/2), workgroup nodes (|up(w)| <=
// 512); longer lists by binary search in global memory
constexpr int kPTriWaveSlots = 128;
constexpr int kPWaves = 16;

template <typename T> struct PersistPool {
  using TW = TriLds<T, kPTriWaveSlots, 64, 64>;
  struct TriWave {
    TW L[kPWaves];
    int2 hq[kPWaves][kQueue];
  };
  using TB = TriBlockLds<T, 2048, 512, kPWaves, 1024>;
  struct Pass2 {
    Pass2Lds L;
    int32_t list[1024];
    int32_t cnt[4];
  };
  static constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
  static constexpr size_t kBytes =
      cmax(cmax(cmax(sizeof(MidLds<T, 1>), (size_t)BigLds<T>::kBytes),
                cmax(sizeof(TriWave), sizeof(TB))),
           sizeof(Pass2));
};

struct PersistArgs {
  const int32_t *row_ptr, *col, *deg;
  const int2 *adj2, *adjs;
  TriArgs tri;
  FinArgs fin;
  void *R, *rec;
  // per-bin lists, each ordered by graph
  const int32_t *pair[7];  // tiny, S16, S32, S64, mid G4, G2, G1 (centre ids)
  const BigCentre *big;
  const TileItem *tiles;
  const int2 *reduce;
  const int4 *tri_lane, *tri_wave;
  const int32_t *tri_block, *tri_long;
  const int32_t *fin_list[4];  // 8-lane, 32-lane, wavefront, workgroup tiers
  // schedule
  const int4 *items;   // {type, graph, a, b}
  int32_t n_items;
  int32_t n_graphs;
  int32_t *ctl;        // [0] cursor, [1] workgroups that left, [2] error flag, [3] pass-2
                       // seeds, [4] FP64-finalised seeds; [8..12] the last launch's
                       // error flag, pass-2 and FP64 counts
  int32_t *pend;       // [3 * n_graphs]: items of phases 0, 1, 2 left per graph
  const int32_t *pend0;
  int32_t spin_limit;
};

// thread 0: wait until graph g has no item of a phase below ph left
__device__ inline bool persist_wait(const PersistArgs &P, int32_t g, int ph) {
  for (int q = 0; q < ph; ++q) {
    int32_t spins = 0;
    while (__hip_atomic_load(&P.pend[3 * g + q], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >
           0) {
      // after an error nothing waits: items whose inputs are missing are dropped
      if (__hip_atomic_load(&P.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if (++spins > P.spin_limit) {
        atomicOr(&P.ctl[2], 1);
        return false;
      }
      __builtin_amdgcn_s_sleep(8);
    }
  }
  return true;
}

template <typename T>
__device__ inline void persist_item(const PersistArgs &P, const int4 it, unsigned char *pool,
                                    int32_t &tab_v) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t type = it.x, a = it.z, b = it.w, cnt = b - a;
  switch (type) {
    case PI_PAIR_LANE:
      for (int32_t i = a + tid; i < b; i += 1024)
        pairs_lane_one<T>(P.row_ptr, P.deg, P.adj2, P.pair[0][i], P.R);
      break;
    case PI_PAIR_S16:
      for (int64_t gi = wv; gi < (cnt + 3) / 4; gi += kPWaves)
        pairs_seg_group<T, 16>(P.row_ptr, P.deg, P.adj2, P.pair[1] + a, cnt, gi, P.R);
      break;
    case PI_PAIR_S32:
      for (int64_t gi = wv; gi < (cnt + 1) / 2; gi += kPWaves)
        pairs_seg_group<T, 32>(P.row_ptr, P.deg, P.adj2, P.pair[2] + a, cnt, gi, P.R);
      break;
    case PI_PAIR_S64:
      for (int64_t gi = wv; gi < cnt; gi += kPWaves)
        pairs_seg_group<T, 64>(P.row_ptr, P.deg, P.adj2, P.pair[3] + a, cnt, gi, P.R);
      break;
    case PI_PAIR_M4:
      for (int64_t gi = 0; gi < (cnt + 3) / 4; ++gi)
        pairs_mid_group<T, 4>(P.row_ptr, P.deg, P.adjs, P.pair[4] + a, cnt, gi, P.R,
                              *reinterpret_cast<MidLds<T, 4> *>(pool));
      break;
    case PI_PAIR_M2:
      for (int64_t gi = 0; gi < (cnt + 1) / 2; ++gi)
        pairs_mid_group<T, 2>(P.row_ptr, P.deg, P.adjs, P.pair[5] + a, cnt, gi, P.R,
                              *reinterpret_cast<MidLds<T, 2> *>(pool));
      break;
    case PI_PAIR_M1:
      for (int64_t gi = 0; gi < cnt; ++gi)
        pairs_mid_group<T, 1>(P.row_ptr, P.deg, P.adjs, P.pair[6] + a, cnt, gi, P.R,
                              *reinterpret_cast<MidLds<T, 1> *>(pool));
      break;
    case PI_PAIR_BIG:
      for (int32_t i = a; i < b; ++i)
        pairs_big_tile<T>(P.row_ptr, P.deg, P.adjs, P.big, P.tiles[i], P.rec, pool, tab_v);
      return;  // the score table stays valid for the next big item
    case PI_TRI_LANE:
      for (int32_t i = a + tid; i < b; i += 1024)
        tri_lane_node<T, kTriLaneM>(P.tri, P.tri_lane[i]);
      break;
    case PI_TRI_WAVE: {
      auto &W = *reinterpret_cast<typename PersistPool<T>::TriWave *>(pool);
      tri_wave_init(W.L[wv]);
      for (int32_t i = a + wv; i < b; i += kPWaves)
        tri_wave_node<T, kPTriWaveSlots, 64>(P.tri, P.tri_wave[i], W.L[wv],
                                            W.hq[wv]);
      __syncthreads();  // the pool is shared: every wavefront is done with it
      break;
    }
    case PI_TRI_BLOCK: {
      auto &B = *reinterpret_cast<typename PersistPool<T>::TB *>(pool);
      tri_block_init(B);
      __syncthreads();
      for (int32_t i = a; i < b; ++i)
        tri_block_node<T, 2048, 512, kPWaves, 1024>(P.tri, P.tri_block[i], B);
      break;
    }
    case PI_TRI_LONG:
      for (int32_t i = a + wv; i < b; i += kPWaves) {
        const int32_t w = P.tri_long[i];
        // its upper-end records take atomic adds: clear them first
        const int32_t w0 = P.tri.up_ptr[w], m = P.tri.up_ptr[w + 1] - w0;
        for (int32_t j = lane; j < m; j += 64) P.tri.Y[w0 + j] = TriSlot{0, 0, 0};
        __threadfence();
        tri_long_node<T>(P.tri, w);
      }
      break;
    case PI_REDUCE:
      for (int32_t i = a; i < b; ++i)
        arc_reduce_item<T>(P.row_ptr, P.deg, P.adjs, P.big, P.reduce[i], P.rec, P.R);
      break;
    case PI_FIN_LANE:
      fin_lanes<T>(P.fin, a, b, 0, 1);
      break;
    case PI_FIN_G8:
      fin_groups<T, 8>(P.fin, P.fin_list[0] + a, cnt, 0, 0, 1);
      break;
    case PI_FIN_G32:
      fin_groups<T, 32>(P.fin, P.fin_list[1] + a, cnt, 0, 0, 1);
      break;
    case PI_FIN_G64:
      fin_groups<T, 64>(P.fin, P.fin_list[2] + a, cnt, 0, 0, 1);
      break;
    case PI_FIN_HUB:
      fin_hubs<T>(P.fin, P.fin_list[3] + a, cnt, 0, 1);
      break;
    case PI_PASS2: {
      // nodes a..b-1: FP32C pass 2 of the flagged ones, one at a time with
      // the whole workgroup; counts of pass-2 and FP64-finalised seeds
      auto &Q = *reinterpret_cast<typename PersistPool<T>::Pass2 *>(pool);
      int32_t n2 = 0, n64 = 0;
      for (int32_t c0 = a; c0 < b; c0 += 1024) {
        const int32_t v = c0 + tid;
        const uint8_t f = v < b ? P.fin.fl[v] : 0;
        n64 += (f >> 1) & 1;
        const bool p2 = f & 1;
        if (tid == 0) Q.cnt[0] = 0;
        __syncthreads();
        if (p2) Q.list[atomicAdd(&Q.cnt[0], 1)] = v;
        __syncthreads();
        const int32_t m = Q.cnt[0];
        n2 += tid == 0 ? m : 0;
        // each seed's result is its own (a fixed-order sum), whatever order
        // the seeds are taken in
        for (int32_t j = 0; j < m; ++j) {
          const int32_t s = Q.list[j];
          pass2_seed(P.row_ptr, P.col, P.deg, P.adj2, s, s, P.fin.ef, P.fin.D, Q.L);
        }
        __syncthreads();
      }
      n64 = wave_sum_i64(n64);
      if (lane == 0 && n64) atomicAdd(&P.ctl[4], (int32_t)n64);
      if (tid == 0 && n2) atomicAdd(&P.ctl[3], n2);
      break;
    }
    default:
      break;
  }
  tab_v = -1;  // another item used the pool
}

template <typename T>
__global__ __launch_bounds__(1024) void k_batch_persist(PersistArgs P) {
  __shared__ __align__(16) unsigned char pool[PersistPool<T>::kBytes];
  __shared__ int32_t s_item, s_ok;
  int32_t tab_v = -1;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&P.ctl[0], 1);
    __syncthreads();
    const int32_t i = s_item;
    if (i >= P.n_items) break;
    const int4 it = P.items[i];
    const int ph = pitem_phase(it.x);
    if (ph > 0) {
      // one device-scope acquire for the workgroup: it invalidates the
      // caches the workgroup reads through (its compute unit's and its
      // XCD's), and the barrier orders every wavefront's reads after it
      if (threadIdx.x == 0) {
        s_ok = persist_wait(P, it.y, ph);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      if (!s_ok) continue;  // uniform: s_ok is shared (error flag raised)
    }
    persist_item<T>(P, it, pool, tab_v);
    // every wavefront waits for its own stores, then one device-scope release
    // (which writes the XCD's cache back) before the item is counted
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0 && ph < 3) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(&P.pend[3 * it.y + ph], -1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  // the last workgroup to leave resets the schedule for the next launch
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int32_t left = atomicAdd(&P.ctl[1], 1);
    if (left == (int32_t)gridDim.x - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      P.ctl[8] = P.ctl[2];
      P.ctl[9] = P.ctl[3];
      P.ctl[10] = P.ctl[4];
      for (int32_t q = 0; q < 3 * P.n_graphs; ++q) P.pend[q] = P.pend0[q];
      P.ctl[0] = 0;
      P.ctl[2] = 0;
      P.ctl[3] = 0;
      P.ctl[4] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      P.ctl[1] = 0;
    }
  }
}

}  // namespace efi

namespace efi {

template <typename T>
static hipError_t persist_impl(const Graph &g, const PersistPlan &pl, void *R, void *rec,
                               TriSlot *Y, void *Z, int64_t *ZT, double *ef, int64_t *D,
                               int64_t *N, uint8_t *fl, hipStream_t st) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persist<T>, 1024, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1 || cus < 1) return hipErrorLaunchOutOfResources;
  PersistArgs P{};
  P.row_ptr = g.row_ptr;
  P.col = g.col_idx;
  P.deg = g.deg;
  P.adj2 = g.adj2;
  P.adjs = g.adjs ? g.adjs : g.adj2;
  P.tri = TriArgs{g.up_ptr, g.up_col, g.up_deg, g.dn_ptr, g.dn, g.nnz / 2, Y, Z, ZT};
  P.fin = FinArgs{g.row_ptr, g.deg, g.adj2, g.rrev, g.trec, g.dn_ptr, g.asum, g.qa,
                  R,         Y,     Z,      ZT,    ef,     D,      N,        fl};
  P.R = R;
  P.rec = rec;
  for (int i = 0; i < 7; ++i) P.pair[i] = pl.pair[i];
  P.big = pl.big;
  P.tiles = pl.tiles;
  P.reduce = pl.reduce;
  P.tri_lane = g.tri_recL;
  P.tri_wave = pl.tri_wave;
  P.tri_block = pl.tri_block;
  P.tri_long = pl.tri_long;
  for (int i = 0; i < 4; ++i) P.fin_list[i] = pl.fin_list[i];
  P.items = pl.items;
  P.n_items = pl.n_items;
  P.n_graphs = pl.n_graphs;
  P.ctl = pl.ctl;
  P.pend = pl.pend;
  P.pend0 = pl.pend0;
  P.spin_limit = kPersistSpinLimit;
  const int64_t grid = std::min<int64_t>((int64_t)per_cu * cus, std::max(pl.n_items, 1));
  hipLaunchKernelGGL(k_batch_persist<T>, dim3((unsigned)grid), dim3(1024), 0, st, P);
  return hipGetLastError();
}

hipError_t launch_batch_persist(const Graph &g, ef_prec prec, const PersistPlan &pl, void *R,
                                void *rec, TriSlot *Y, void *Z, int64_t *ZT, double *ef,
                                int64_t *D, int64_t *N, uint8_t *fl, hipStream_t st) {
  if (pl.n_items <= 0) return hipSuccess;
  if (prec == EF_PREC_FP64) return persist_impl<double>(g, pl, R, rec, Y, Z, ZT, ef, D, N, fl, st);
  return persist_impl<float>(g, pl, R, rec, Y, Z, ZT, ef, D, N, fl, st);
}

}  // namespace efi
