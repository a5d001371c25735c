// Batched Expected Force: many graphs in one pass.
//
// The graphs are loaded as one disjoint union. A cluster never spans two
// components, so the EF of every node in the union equals its EF in its own
// graph, and every phase of the exact path (binning, pair loops, triangle
// pass, per-node sums, pass 2) runs once over all graphs: one launch per
// phase covers the whole batch, with one shared work list per degree bin.
//
// The launch sequence of one batch computation is captured once into a HIP
// graph on a private stream and replayed by every later call. The small-bin
// segment thresholds are chosen by timing the candidates on the batch itself
// (ef_batch_autotune, run on first use).
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "ef_internal.h"

extern "C" ef_status ef_compute(ef_graph *g, ef_algo algo, ef_prec prec, const int32_t *seeds,
                                int32_t n_seeds, double *ef, int64_t *D, int64_t *N,
                                uint32_t flags, void *hip_stream);
extern "C" ef_status ef_graph_load_csr(int32_t n, int64_t nnz, const int32_t *row_ptr,
                                       const int32_t *col_idx, uint32_t flags, void *hip_stream,
                                       ef_graph **out);
extern "C" ef_status ef_graph_free(ef_graph *g);
extern "C" ef_status ef_validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr,
                                     const int32_t *col_idx);


namespace efi {

// candidate small-bin thresholds (t8, t16, t32)
static const SmallThr kCandidates[] = {
    {8, 16, 32}, {0, 16, 32}, {8, 0, 32}, {8, 16, 0}, {0, 0, 32}, {0, 16, 0}, {0, 0, 0}, {8, 0, 0},
};
}  // namespace efi

using namespace efi;

struct ef_batch {
  ef_graph *g = nullptr;
  int32_t n_graphs = 0;
  int32_t n = 0;
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool captured = false;
  ef_prec cap_prec = EF_PREC_FP32C;
  bool tuned = false;
  double *ef_s = nullptr;
  int64_t *D_s = nullptr, *N_s = nullptr;
  ef_batch_stats stats{};
};

static void drop_graph(ef_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->captured = false;
}

extern "C" ef_status ef_batch_free(ef_batch *b) {
  if (!b) {
    set_error("ef_batch_free: null handle");
    return EF_ERR_ARG;
  }
  drop_graph(b);
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
  ef_status s = ef_graph_load_csr(n, nnz, row_ptr, col_idx, 0, hip_stream, &b->g);
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

// one eager pass on the private stream into the staging buffers, timed
static ef_status eager(ef_batch *b, ef_prec prec, float *ms) {
  hipError_t e = hipEventRecord(b->t0, b->own);
  if (e != hipSuccess) return hip_status(e, "event");
  ef_status s = ef_compute(b->g, EF_ALGO_CLUSTER, prec, nullptr, 0, b->ef_s, b->D_s, b->N_s,
                           EF_OUT_DEVICE | kInternalNoReadback, b->own);
  if (s != EF_OK) return s;
  e = hipEventRecord(b->t1, b->own);
  if (e == hipSuccess) e = hipEventSynchronize(b->t1);
  if (e == hipSuccess && ms) e = hipEventElapsedTime(ms, b->t0, b->t1);
  return hip_status(e, "eager batch pass");
}

extern "C" ef_status ef_batch_autotune(ef_batch *b, ef_prec prec) {
  if (!b || (prec != EF_PREC_FP64 && prec != EF_PREC_FP32C)) {
    set_error("ef_batch_autotune: bad arguments");
    return EF_ERR_ARG;
  }
  Graph &g = b->g->g;
  const SmallThr keep = g.thr;
  float best = 1e30f;
  SmallThr best_thr = keep;
  int idx = 0, best_idx = 0;
  for (const SmallThr &c : kCandidates) {
    g.thr = c;
    float t = 0.f, tmin = 1e30f;
    ef_status s = eager(b, prec, &t);  // warm-up (also sizes the workspace)
    for (int r = 0; r < 3 && s == EF_OK; ++r) {
      s = eager(b, prec, &t);
      tmin = std::min(tmin, t);
    }
    if (s != EF_OK) {
      g.thr = keep;
      return s;
    }
    if (idx < 8) b->stats.tune_ms[idx] = tmin;
    if (tmin < best) {
      best = tmin;
      best_thr = c;
      best_idx = idx;
    }
    ++idx;
  }
  g.thr = best_thr;
  b->tuned = true;
  b->stats.tuned_choice = best_idx;
  b->stats.thr8 = best_thr.t8;
  b->stats.thr16 = best_thr.t16;
  b->stats.thr32 = best_thr.t32;
  drop_graph(b);
  return EF_OK;
}

static ef_status capture(ef_batch *b, ef_prec prec) {
  drop_graph(b);
  // an eager pass first: sizes every workspace buffer, so nothing is
  // allocated while the stream is being captured
  ef_status s = eager(b, prec, nullptr);
  if (s != EF_OK) return s;
  hipError_t e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_status(e, "begin capture");
  s = ef_compute(b->g, EF_ALGO_CLUSTER, prec, nullptr, 0, b->ef_s, b->D_s, b->N_s,
                 EF_OUT_DEVICE | kInternalNoReadback, b->own);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(b->own, &graph);
  if (s != EF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return hip_status(e, "end capture");
  b->graph = graph;
  e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return hip_status(e, "instantiate graph");
  }
  b->captured = true;
  b->cap_prec = prec;
  return EF_OK;
}

extern "C" ef_status ef_batch_compute(ef_batch *b, ef_prec prec, double *ef, int64_t *D,
                                      int64_t *N, uint32_t flags, void *hip_stream) {
  if (!b || !ef || (prec != EF_PREC_FP64 && prec != EF_PREC_FP32C)) {
    set_error("ef_batch_compute: bad arguments");
    return EF_ERR_ARG;
  }
  if (flags & ~(EF_OUT_DEVICE | EF_PROFILE)) {
    set_error("ef_batch_compute: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  if (b->n == 0) return EF_OK;
  ef_status s;
  if (!b->tuned && (s = ef_batch_autotune(b, prec)) != EF_OK) return s;
  if (!b->captured || b->cap_prec != prec) {
    if ((s = capture(b, prec)) != EF_OK) return s;
  }
  hipStream_t user = (hipStream_t)hip_stream;
  hipError_t e = hipEventRecord(b->ev_in, user);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->own, b->ev_in, 0);
  if (e == hipSuccess) e = hipEventRecord(b->t0, b->own);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->own);
  if (e == hipSuccess) e = hipEventRecord(b->t1, b->own);
  const size_t nn = (size_t)b->n;
  const hipMemcpyKind kind =
      (flags & EF_OUT_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (e == hipSuccess) e = hipMemcpyAsync(ef, b->ef_s, sizeof(double) * nn, kind, b->own);
  if (e == hipSuccess && D) e = hipMemcpyAsync(D, b->D_s, sizeof(int64_t) * nn, kind, b->own);
  if (e == hipSuccess && N) e = hipMemcpyAsync(N, b->N_s, sizeof(int64_t) * nn, kind, b->own);
  if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->own);
  if (e == hipSuccess) e = hipStreamWaitEvent(user, b->ev_out, 0);
  if (e == hipSuccess && (!(flags & EF_OUT_DEVICE) || (flags & EF_PROFILE)))
    e = hipStreamSynchronize(b->own);
  if (e == hipSuccess && (flags & EF_PROFILE)) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, b->t0, b->t1);
    b->stats.replay_ms = ms;
  }
  return hip_status(e, "batch replay");
}

extern "C" ef_status ef_batch_stats_get(const ef_batch *b, ef_batch_stats *out) {
  if (!b || !out) {
    set_error("ef_batch_stats_get: null argument");
    return EF_ERR_ARG;
  }
  *out = b->stats;
  return EF_OK;
}
