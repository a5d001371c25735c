// Batched Expected Force: many graphs in one pass.
//
// The graphs are loaded as one disjoint union. A cluster never spans two
// components, so the EF of every node in the union equals its EF in its own
// graph. Two designs compute the union:
//
//   phased      every phase of the exact path (binning, pair loops, triangle
//               pass, per-node sums, pass 2) runs once over all graphs, one
//               launch per phase and bin, with one shared work list per
//               degree bin;
//   persistent  one launch of a persistent kernel (exact/batch_persist.hip)
//               whose workgroups take (graph, bin, chunk) items from an atomic
//               cursor, each graph moving to its next phase as soon as its own
//               items of the previous one are done.
//
// Either launch sequence is captured once into a HIP graph on a private
// stream and replayed by every later call. ef_batch_autotune times both
// designs on the batch itself, each with several settings (small-bin segment
// thresholds; for the persistent design also the chunk size of its items),
// keeps the fastest and caches the choice per size class (graph count, nodes,
// arcs and largest degree, each rounded to a power of two), so later batches
// of the same class skip the timing.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "ef_internal.h"

extern "C" ef_status ef_compute(ef_graph *g, ef_algo algo, ef_prec prec, const int32_t *seeds,
                                int32_t n_seeds, double *ef, int64_t *D, int64_t *N,
                                uint32_t flags, void *hip_stream);
extern "C" ef_status ef_graph_free(ef_graph *g);
extern "C" ef_status ef_validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr,
                                     const int32_t *col_idx);

namespace efi {

// candidate small-bin thresholds (t8, t16, t32) of the phased design
static const SmallThr kCandidates[] = {
    {8, 16, 32}, {0, 16, 32}, {8, 0, 32}, {8, 16, 0}, {0, 0, 32}, {0, 16, 0}, {0, 0, 0}, {8, 0, 0},
};

// settings of the persistent design: small-bin thresholds and the chunk
// size of the items (a multiple of the base sizes below)
struct PersistCfg {
  SmallThr thr;
  int32_t scale;
};
static const PersistCfg kPersistCandidates[] = {
    {{8, 16, 32}, 1},  {{8, 16, 32}, 4}, {{8, 16, 32}, 16}, {{8, 16, 32}, 64},
    {{8, 0, 32}, 16},  {{0, 16, 32}, 16}, {{8, 16, 0}, 16}, {{8, 0, 0}, 16},
};

// base chunk of each item type (entries of its list, or node ids)
static int32_t item_chunk(int32_t type, int32_t scale) {
  switch (type) {
    case PI_PAIR_LANE: return 2048 * scale;
    case PI_PAIR_S16: return 128 * scale;
    case PI_PAIR_S32: return 64 * scale;
    case PI_PAIR_S64: return 32 * scale;
    case PI_PAIR_M4: return 16 * scale;
    case PI_PAIR_M2: return 8 * scale;
    case PI_PAIR_M1: return 2 * scale;
    case PI_TRI_LANE: return 2048 * scale;
    case PI_TRI_WAVE: return 32 * scale;
    case PI_TRI_LONG: return 16;
    case PI_REDUCE: return 2;
    case PI_FIN_LANE: return 4096 * scale;
    case PI_FIN_G8: return 512 * scale;
    case PI_FIN_G32: return 128 * scale;
    case PI_FIN_G64: return 32 * scale;
    case PI_FIN_HUB: return 2;
    case PI_PASS2: return 8192 * scale;
    default: return 1;  // big tiles, workgroup triangle nodes
  }
}

// the tuning of one size class and precision, shared by every batch of the
// process
struct TuneEntry {
  SmallThr thr;
  int32_t phased_choice, persist_choice, design;
};
static std::mutex g_tune_mu;
static std::map<int64_t, TuneEntry> g_tune_cache;

}  // namespace efi

using namespace efi;

// device memory of the persistent design
struct PersistState {
  PersistPlan pl;
  std::vector<void *> owned;
  void *R = nullptr, *rec = nullptr, *Z = nullptr;
  TriSlot *Y = nullptr;
  int64_t *ZT = nullptr;
  uint8_t *fl = nullptr;
  int32_t cfg = -1;  // candidate the plan was built for
};

struct ef_batch {
  ef_graph *g = nullptr;
  int32_t n_graphs = 0;
  int32_t n = 0;
  std::vector<int64_t> node_off;
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
  // captured launch sequence per design (0 phased, 1 persistent)
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  ef_prec cap_prec[2] = {EF_PREC_FP32C, EF_PREC_FP32C};
  bool tuned = false;
  int32_t design = 0;
  int32_t persist_cfg = 0;
  PersistState ps;
  double *ef_s = nullptr;
  int64_t *D_s = nullptr, *N_s = nullptr;
  ef_batch_stats stats{};
};

static void drop_graph(ef_batch *b, int d) {
  if (b->exec[d]) (void)hipGraphExecDestroy(b->exec[d]);
  if (b->graph[d]) (void)hipGraphDestroy(b->graph[d]);
  b->exec[d] = nullptr;
  b->graph[d] = nullptr;
}

static void drop_persist(ef_batch *b) {
  drop_graph(b, 1);
  for (void *p : b->ps.owned) (void)hipFree(p);
  b->ps = PersistState{};
}

extern "C" ef_status ef_batch_free(ef_batch *b) {
  if (!b) {
    set_error("ef_batch_free: null handle");
    return EF_ERR_ARG;
  }
  drop_graph(b, 0);
  drop_persist(b);
  if (b->ef_s) (void)hipFree(b->ef_s);
  if (b->D_s) (void)hipFree(b->D_s);
  if (b->N_s) (void)hipFree(b->N_s);
  for (hipEvent_t e : {b->ev_in, b->ev_out, b->t0, b->t1})
    if (e) (void)hipEventDestroy(e);
  if (b->own) (void)hipStreamDestroy(b->own);
  if (b->g) ef_graph_free(b->g);
  delete b;
  return EF_OK;
}

extern "C" ef_status ef_batch_create(int32_t n_graphs, const int32_t *node_off, int64_t nnz,
                                     const int32_t *row_ptr, const int32_t *col_idx,
                                     uint32_t flags, void *hip_stream, ef_batch **out) {
  if (!out || n_graphs < 0 || !node_off || !row_ptr || (nnz > 0 && !col_idx)) {
    set_error("ef_batch_create: bad arguments");
    return EF_ERR_ARG;
  }
  *out = nullptr;
  if (flags & ~EF_VALIDATE) {
    set_error("ef_batch_create: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  if (node_off[0] != 0) {
    set_error("ef_batch_create: node_off[0] must be 0");
    return EF_ERR_RANGE;
  }
  for (int32_t i = 0; i < n_graphs; ++i)
    if (node_off[i + 1] < node_off[i]) {
      set_error("ef_batch_create: node_off decreases at graph %d", i);
      return EF_ERR_UNSORTED;
    }
  const int32_t n = node_off[n_graphs];
  if (flags & EF_VALIDATE) {
    ef_status s = ef_validate_csr(n, nnz, row_ptr, col_idx);
    if (s != EF_OK) return s;
    for (int32_t gi = 0; gi < n_graphs; ++gi)
      for (int32_t v = node_off[gi]; v < node_off[gi + 1]; ++v)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
          if (col_idx[e] < node_off[gi] || col_idx[e] >= node_off[gi + 1]) {
            set_error("arc %d->%d leaves graph %d", v, col_idx[e], gi);
            return EF_ERR_RANGE;
          }
  }
  ef_batch *b = new (std::nothrow) ef_batch();
  if (!b) {
    set_error("host allocation failed");
    return EF_ERR_NOMEM;
  }
  b->n_graphs = n_graphs;
  b->n = n;
  b->node_off.assign(node_off, node_off + n_graphs + 1);
  ef_status s = graph_load(n, nnz, row_ptr, col_idx, 0, hip_stream, b->node_off.data(), n_graphs,
                           &b->g);
  if (s != EF_OK) {
    delete b;
    return s;
  }
  hipError_t e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking);
  for (hipEvent_t *ev : {&b->ev_in, &b->ev_out})
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  for (hipEvent_t *ev : {&b->t0, &b->t1})
    if (e == hipSuccess) e = hipEventCreate(ev);
  const size_t nn = (size_t)std::max(n, 1);
  if (e == hipSuccess) e = hipMalloc(&b->ef_s, sizeof(double) * nn);
  if (e == hipSuccess) e = hipMalloc(&b->D_s, sizeof(int64_t) * nn);
  if (e == hipSuccess) e = hipMalloc(&b->N_s, sizeof(int64_t) * nn);
  if (e != hipSuccess) {
    ef_batch_free(b);
    return hip_status(e, "batch resources");
  }
  b->stats.n_graphs = n_graphs;
  b->stats.n = n;
  b->stats.nnz = nnz;
  b->stats.clusters = b->g->g.info.clusters;
  *out = b;
  return EF_OK;
}

// ---------------------------------------------------------------------------
// persistent design: the schedule
// ---------------------------------------------------------------------------

// offsets per graph of a list of node ids ordered graph by graph; false if
// the list is not in that order
static bool split_by_graph(const ef_batch *b, const int32_t *ids, int64_t count,
                           std::vector<int64_t> &off) {
  off.assign((size_t)b->n_graphs + 1, 0);
  int32_t gi = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int32_t v = ids[i];
    if (v < b->node_off[gi]) return false;
    while (gi < b->n_graphs && v >= b->node_off[gi + 1]) off[(size_t)++gi] = i;
    if (gi >= b->n_graphs) return false;
  }
  while (gi < b->n_graphs) off[(size_t)++gi] = count;
  return true;
}

template <typename V>
static ef_status upload(PersistState &ps, const std::vector<V> &h, V **out, const char *what) {
  *out = nullptr;
  const size_t bytes = sizeof(V) * std::max<size_t>(h.size(), 1);
  hipError_t e = hipMalloc((void **)out, bytes);
  if (e == hipSuccess) {
    ps.owned.push_back(*out);
    if (!h.empty()) e = hipMemcpy(*out, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice);
  }
  return hip_status(e, what);
}

static ef_status dev_buffer(PersistState &ps, size_t bytes, void **out, const char *what) {
  hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 256));
  if (e == hipSuccess) ps.owned.push_back(*out);
  return hip_status(e, what);
}

static ef_status build_persist(ef_batch *b, int32_t cfg_idx) {
  drop_persist(b);
  const PersistCfg cfg = kPersistCandidates[cfg_idx];
  Graph &g = b->g->g;
  const int32_t G = b->n_graphs;
  PersistState &ps = b->ps;
  // pair bins, graph by graph
  std::vector<int32_t> pl[7];
  std::vector<int64_t> po[7];
  for (auto &o : po) o.assign((size_t)G + 1, 0);
  std::vector<BigCentre> big;
  std::vector<TileItem> tiles;
  std::vector<int2> red;
  std::vector<int64_t> tile_off((size_t)G + 1, 0), red_off((size_t)G + 1, 0);
  int64_t rec_base = 0;
  for (int32_t gi = 0; gi < G; ++gi) {
    for (int64_t v = b->node_off[gi]; v < b->node_off[gi + 1]; ++v) {
      const int32_t k = g.h_deg[(size_t)v];
      if (k < 2) continue;
      if (k <= kSmallMax) {
        pl[small_bin(k, cfg.thr)].push_back((int32_t)v);
      } else if (k <= kSuper) {
        pl[4 + mid_class(k)].push_back((int32_t)v);
      } else {
        const int32_t ns = (k + kSuper - 1) / kSuper;
        const int32_t bi = (int32_t)big.size();
        big.push_back(BigCentre{(int32_t)v, ns, rec_base});
        for (int32_t P = 0; P < ns; ++P) {
          for (int32_t Q = P; Q < ns; ++Q) tiles.push_back(TileItem{bi, P, Q});
          red.push_back(make_int2(bi, P));
        }
        rec_base += (int64_t)ns * (ns + 1) / 2;
      }
    }
    for (int q = 0; q < 7; ++q) po[q][(size_t)gi + 1] = (int64_t)pl[q].size();
    tile_off[(size_t)gi + 1] = (int64_t)tiles.size();
    red_off[(size_t)gi + 1] = (int64_t)red.size();
  }
  // triangle and finalize lists of the union, already graph by graph
  std::vector<int64_t> tl_off, tw_off, tb_off, t2_off, t3_off, fh_off, fw_off, fc_off, fg_off;
  const int64_t nf = g.n_fin, nfh = g.n_fin_hub, nfc = g.n_fin_half;
  bool ok = split_by_graph(b, g.h_tri_lane.data(), (int64_t)g.h_tri_lane.size(), tl_off) &&
            split_by_graph(b, g.h_tri[0].data(), (int64_t)g.h_tri[0].size(), tw_off) &&
            split_by_graph(b, g.h_tri[1].data(), (int64_t)g.h_tri[1].size(), tb_off) &&
            split_by_graph(b, g.h_tri[2].data(), (int64_t)g.h_tri[2].size(), t2_off) &&
            split_by_graph(b, g.h_tri[3].data(), (int64_t)g.h_tri[3].size(), t3_off) &&
            split_by_graph(b, g.h_fin.data(), nfh, fh_off) &&
            split_by_graph(b, g.h_fin.data() + nfh, nf - nfh - nfc, fw_off) &&
            split_by_graph(b, g.h_fin.data() + nf - nfc, nfc, fc_off) &&
            split_by_graph(b, g.h_fin.data() + nf, g.n_fin_group, fg_off);
  if (!ok) {
    set_error("persistent batch: node lists are not ordered graph by graph");
    return EF_ERR_STATE;
  }
  // long triangle lists (bins 2 and 3), graph by graph
  std::vector<int32_t> tlong;
  std::vector<int64_t> tg_off((size_t)G + 1, 0);
  for (int32_t gi = 0; gi < G; ++gi) {
    tlong.insert(tlong.end(), g.h_tri[2].begin() + t2_off[gi], g.h_tri[2].begin() + t2_off[gi + 1]);
    tlong.insert(tlong.end(), g.h_tri[3].begin() + t3_off[gi], g.h_tri[3].begin() + t3_off[gi + 1]);
    tg_off[(size_t)gi + 1] = (int64_t)tlong.size();
  }
  // items: phase 0 heaviest bins first, every phase graph by graph
  std::vector<int4> items;
  std::vector<int32_t> pend0((size_t)3 * G, 0);
  auto add_items = [&](int32_t type, const std::vector<int64_t> &off, int64_t base) {
    const int64_t chunk = item_chunk(type, cfg.scale);
    const int ph = pitem_phase(type);
    for (int32_t gi = 0; gi < G; ++gi)
      for (int64_t a = off[gi]; a < off[gi + 1]; a += chunk) {
        items.push_back(make_int4(type, gi, (int32_t)(base + a),
                                  (int32_t)(base + std::min(off[gi + 1], a + chunk))));
        if (ph < 3) pend0[(size_t)3 * gi + ph]++;
      }
  };
  add_items(PI_PAIR_BIG, tile_off, 0);
  add_items(PI_TRI_LONG, tg_off, 0);
  add_items(PI_TRI_BLOCK, tb_off, 0);
  add_items(PI_PAIR_M1, po[6], 0);
  add_items(PI_PAIR_M2, po[5], 0);
  add_items(PI_PAIR_M4, po[4], 0);
  add_items(PI_TRI_WAVE, tw_off, 0);
  add_items(PI_PAIR_S64, po[3], 0);
  add_items(PI_PAIR_S32, po[2], 0);
  add_items(PI_PAIR_S16, po[1], 0);
  add_items(PI_PAIR_LANE, po[0], 0);
  add_items(PI_TRI_LANE, tl_off, 0);
  add_items(PI_REDUCE, red_off, 0);
  // finalize tiers index the union's fin_list: hubs at 0, wavefront tier
  // after them, 32-lane tier before n_fin, 8-lane tier from n_fin
  {
    std::vector<int4> fin_items;
    const size_t first = items.size();
    add_items(PI_FIN_HUB, fh_off, 0);
    add_items(PI_FIN_G64, fw_off, 0);
    add_items(PI_FIN_G32, fc_off, 0);
    add_items(PI_FIN_G8, fg_off, 0);
    add_items(PI_FIN_LANE, b->node_off, 0);
    // graph by graph across the tiers
    std::stable_sort(items.begin() + (int64_t)first, items.end(),
                     [](const int4 &x, const int4 &y) { return x.y < y.y; });
  }
  add_items(PI_PASS2, b->node_off, 0);
  if (items.size() >= (size_t)INT32_MAX) {
    set_error("persistent batch: too many work items");
    return EF_ERR_OVERFLOW;
  }
  ef_status s = EF_OK;
  PersistPlan &P = ps.pl;
  for (int q = 0; q < 7 && s == EF_OK; ++q) s = upload(ps, pl[q], &P.pair[q], "pair lists");
  if (s == EF_OK) s = upload(ps, big, &P.big, "big centres");
  if (s == EF_OK) s = upload(ps, tiles, &P.tiles, "super-tiles");
  if (s == EF_OK) s = upload(ps, red, &P.reduce, "reduction items");
  if (s == EF_OK) s = upload(ps, tlong, &P.tri_long, "long triangle nodes");
  if (s == EF_OK) s = upload(ps, items, &P.items, "work items");
  if (s == EF_OK) s = upload(ps, pend0, &P.pend0, "item counts");
  if (s == EF_OK) s = upload(ps, pend0, &P.pend, "item counters");
  if (s == EF_OK) s = upload(ps, std::vector<int32_t>(16, 0), &P.ctl, "cursor");
  if (s != EF_OK) return s;
  P.tri_wave = g.tri_rec0;
  P.tri_block = g.tri_list[1];
  P.fin_list[0] = g.fin_list + nf;
  P.fin_list[1] = g.fin_list + (nf - nfc);
  P.fin_list[2] = g.fin_list + nfh;
  P.fin_list[3] = g.fin_list;
  P.n_items = (int32_t)items.size();
  P.n_graphs = G;
  // workspace; R and the records hold float2 or double: 8 bytes either way
  const size_t nnz = (size_t)std::max<int64_t>(g.nnz, 1), n = (size_t)std::max(g.n, 1);
  if (s == EF_OK) s = dev_buffer(ps, 8 * nnz, &ps.R, "arc sums");
  if (s == EF_OK)
    s = dev_buffer(ps, (size_t)8 * kRecEntries * (size_t)std::max<int64_t>(rec_base, 1), &ps.rec,
                   "super-tile records");
  if (s == EF_OK) s = dev_buffer(ps, sizeof(TriSlot) * nnz, (void **)&ps.Y, "triangle records");
  if (s == EF_OK) s = dev_buffer(ps, 8 * n, &ps.Z, "triangle node sums");
  if (s == EF_OK) s = dev_buffer(ps, 8 * n, (void **)&ps.ZT, "triangle node counts");
  if (s == EF_OK) s = dev_buffer(ps, n, (void **)&ps.fl, "flag bytes");
  if (s != EF_OK) return s;
  ps.cfg = cfg_idx;
  b->stats.items = P.n_items;
  return EF_OK;
}

// one persistent launch into the staging outputs (asynchronous on b->own)
static ef_status launch_persist(ef_batch *b, ef_prec prec) {
  PersistState &ps = b->ps;
  hipError_t e = launch_batch_persist(b->g->g, prec, ps.pl, ps.R, ps.rec, ps.Y, ps.Z, ps.ZT,
                                      b->ef_s, b->D_s, b->N_s, ps.fl, b->own);
  return hip_status(e, "persistent batch kernel");
}

// the last persistent launch's error flag and counts (synchronises b->own)
static ef_status read_persist_result(ef_batch *b) {
  int32_t r[3] = {0, 0, 0};
  hipError_t e = hipMemcpyAsync(r, b->ps.pl.ctl + 8, sizeof(r), hipMemcpyDeviceToHost, b->own);
  if (e == hipSuccess) e = hipStreamSynchronize(b->own);
  if (e != hipSuccess) return hip_status(e, "persistent batch result");
  b->stats.persist_pass2 = r[1];
  b->stats.persist_fp64 = r[2];
  if (r[0]) {
    set_error("persistent batch kernel: a wait for a graph's earlier phase exceeded its limit");
    return EF_ERR_DEVICE;
  }
  return EF_OK;
}

// ---------------------------------------------------------------------------
// timing and tuning
// ---------------------------------------------------------------------------

// one eager pass of a design on the private stream into the staging buffers
static ef_status eager(ef_batch *b, int design, ef_prec prec, float *ms) {
  hipError_t e = hipEventRecord(b->t0, b->own);
  if (e != hipSuccess) return hip_status(e, "event");
  ef_status s;
  if (design == 1) {
    s = launch_persist(b, prec);
  } else {
    s = ef_compute(b->g, EF_ALGO_CLUSTER, prec, nullptr, 0, b->ef_s, b->D_s, b->N_s,
                   EF_OUT_DEVICE | kInternalNoReadback, b->own);
  }
  if (s != EF_OK) return s;
  e = hipEventRecord(b->t1, b->own);
  if (e == hipSuccess) e = hipEventSynchronize(b->t1);
  if (e == hipSuccess && ms) e = hipEventElapsedTime(ms, b->t0, b->t1);
  if (e != hipSuccess) return hip_status(e, "eager batch pass");
  return design == 1 ? read_persist_result(b) : EF_OK;
}

static float time_design(ef_batch *b, int design, ef_prec prec, ef_status &s) {
  float t = 0.f, tmin = 1e30f;
  s = eager(b, design, prec, &t);  // warm-up
  for (int r = 0; r < 3 && s == EF_OK; ++r) {
    s = eager(b, design, prec, &t);
    tmin = std::min(tmin, t);
  }
  return tmin;
}

static int64_t size_class(ef_batch *b, ef_prec prec) {
  auto lg = [](int64_t x) {
    int64_t r = 0;
    while ((1ll << r) < x) ++r;
    return r;
  };
  const Graph &g = b->g->g;
  const int64_t c = (lg(b->n_graphs) << 24) | (lg(g.n) << 16) | (lg(g.nnz) << 8) |
                    lg((int64_t)g.info.max_degree + 1);
  b->stats.size_class = (int32_t)c;
  return 2 * c + (prec == EF_PREC_FP64 ? 1 : 0);
}

static void apply_tuning(ef_batch *b, const TuneEntry &t) {
  Graph &g = b->g->g;
  g.thr = t.thr;
  b->stats.tuned_choice = t.phased_choice;
  b->stats.thr8 = t.thr.t8;
  b->stats.thr16 = t.thr.t16;
  b->stats.thr32 = t.thr.t32;
  b->persist_cfg = t.persist_choice;
  b->stats.persist_choice = t.persist_choice;
  b->design = t.design;
  b->stats.design = t.design;
  b->tuned = true;
}

extern "C" ef_status ef_batch_autotune(ef_batch *b, ef_prec prec) {
  if (!b || (prec != EF_PREC_FP64 && prec != EF_PREC_FP32C)) {
    set_error("ef_batch_autotune: bad arguments");
    return EF_ERR_ARG;
  }
  drop_graph(b, 0);
  drop_graph(b, 1);
  const int64_t key = size_class(b, prec);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      apply_tuning(b, it->second);
      b->stats.from_cache = 1;
      return EF_OK;
    }
  }
  b->stats.from_cache = 0;
  Graph &g = b->g->g;
  ef_status s = EF_OK;
  // phased design: small-bin thresholds
  TuneEntry best{g.thr, 0, 0, 0};
  float best_phased = 1e30f;
  for (int i = 0; i < 8; ++i) {
    g.thr = kCandidates[i];
    const float t = time_design(b, 0, prec, s);
    if (s != EF_OK) return s;
    b->stats.tune_ms[i] = t;
    if (t < best_phased) {
      best_phased = t;
      best.thr = kCandidates[i];
      best.phased_choice = i;
    }
  }
  g.thr = best.thr;
  // persistent design: thresholds and chunk sizes
  float best_persist = 1e30f;
  for (int i = 0; i < 8; ++i) {
    if ((s = build_persist(b, i)) != EF_OK) return s;
    const float t = time_design(b, 1, prec, s);
    if (s != EF_OK) return s;
    b->stats.persist_tune_ms[i] = t;
    if (t < best_persist) {
      best_persist = t;
      best.persist_choice = i;
    }
  }
  best.design = best_persist < best_phased ? 1 : 0;
  apply_tuning(b, best);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = best;
  }
  return EF_OK;
}

// ---------------------------------------------------------------------------
// capture and replay
// ---------------------------------------------------------------------------
static ef_status capture(ef_batch *b, int design, ef_prec prec) {
  drop_graph(b, design);
  if (design == 1 && b->ps.cfg != b->persist_cfg) {
    ef_status s = build_persist(b, b->persist_cfg);
    if (s != EF_OK) return s;
  }
  // an eager pass first: sizes every workspace buffer, so nothing is
  // allocated while the stream is being captured
  ef_status s = eager(b, design, prec, nullptr);
  if (s != EF_OK) return s;
  hipError_t e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_status(e, "begin capture");
  if (design == 1) {
    s = launch_persist(b, prec);
  } else {
    s = ef_compute(b->g, EF_ALGO_CLUSTER, prec, nullptr, 0, b->ef_s, b->D_s, b->N_s,
                   EF_OUT_DEVICE | kInternalNoReadback, b->own);
  }
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(b->own, &graph);
  if (s != EF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return hip_status(e, "end capture");
  b->graph[design] = graph;
  e = hipGraphInstantiate(&b->exec[design], graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b, design);
    return hip_status(e, "instantiate graph");
  }
  b->cap_prec[design] = prec;
  return EF_OK;
}

extern "C" ef_status ef_batch_compute(ef_batch *b, ef_prec prec, double *ef, int64_t *D,
                                      int64_t *N, uint32_t flags, void *hip_stream) {
  if (!b || !ef || (prec != EF_PREC_FP64 && prec != EF_PREC_FP32C)) {
    set_error("ef_batch_compute: bad arguments");
    return EF_ERR_ARG;
  }
  if (flags & ~(EF_OUT_DEVICE | EF_PROFILE | EF_BATCH_PHASED | EF_BATCH_PERSISTENT)) {
    set_error("ef_batch_compute: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  if ((flags & EF_BATCH_PHASED) && (flags & EF_BATCH_PERSISTENT)) {
    set_error("ef_batch_compute: EF_BATCH_PHASED and EF_BATCH_PERSISTENT together");
    return EF_ERR_ARG;
  }
  if (b->n == 0) return EF_OK;
  const bool forced = (flags & (EF_BATCH_PHASED | EF_BATCH_PERSISTENT)) != 0;
  ef_status s;
  if (!b->tuned && !forced && (s = ef_batch_autotune(b, prec)) != EF_OK) return s;
  const int design = (flags & EF_BATCH_PHASED)       ? 0
                     : (flags & EF_BATCH_PERSISTENT) ? 1
                                                     : b->design;
  if (!b->exec[design] || b->cap_prec[design] != prec) {
    if ((s = capture(b, design, prec)) != EF_OK) return s;
  }
  hipStream_t user = (hipStream_t)hip_stream;
  hipError_t e = hipEventRecord(b->ev_in, user);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->own, b->ev_in, 0);
  if (e == hipSuccess) e = hipEventRecord(b->t0, b->own);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec[design], b->own);
  if (e == hipSuccess) e = hipEventRecord(b->t1, b->own);
  const size_t nn = (size_t)b->n;
  const hipMemcpyKind kind =
      (flags & EF_OUT_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (e == hipSuccess) e = hipMemcpyAsync(ef, b->ef_s, sizeof(double) * nn, kind, b->own);
  if (e == hipSuccess && D) e = hipMemcpyAsync(D, b->D_s, sizeof(int64_t) * nn, kind, b->own);
  if (e == hipSuccess && N) e = hipMemcpyAsync(N, b->N_s, sizeof(int64_t) * nn, kind, b->own);
  if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->own);
  if (e == hipSuccess) e = hipStreamWaitEvent(user, b->ev_out, 0);
  const bool sync = !(flags & EF_OUT_DEVICE) || (flags & EF_PROFILE);
  if (e == hipSuccess && sync) e = hipStreamSynchronize(b->own);
  if (e == hipSuccess && (flags & EF_PROFILE)) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, b->t0, b->t1);
    b->stats.replay_ms = ms;
  }
  if (e != hipSuccess) return hip_status(e, "batch replay");
  if (design == 1 && sync) return read_persist_result(b);
  return EF_OK;
}

extern "C" ef_status ef_batch_stats_get(const ef_batch *b, ef_batch_stats *out) {
  if (!b || !out) {
    set_error("ef_batch_stats_get: null argument");
    return EF_ERR_ARG;
  }
  *out = b->stats;
  return EF_OK;
}
