// C-ABI of the Expected Force library: argument checks, CSR validation, graph
// loading, workspace management and the launch sequence of each entry point.
// All arithmetic of the method runs in the kernels of the .hip files.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "csr_check.h"
#include "ef_internal.h"


namespace efi {

static thread_local std::string t_err;

void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
}

ef_status hip_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return EF_OK;
  set_error("%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return EF_ERR_NOMEM;
  return EF_ERR_DEVICE;
}

static int64_t max_device_bytes() {
  const char *s = std::getenv("EF_MAX_DEVICE_BYTES");
  if (!s || !*s) return INT64_MAX;
  char *end = nullptr;
  long long v = std::strtoll(s, &end, 10);
  return v > 0 ? (int64_t)v : INT64_MAX;
}

// allocation accounted against EF_MAX_DEVICE_BYTES
static ef_status dev_alloc(Graph &g, void **p, size_t bytes, const char *what) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (g.owned_bytes + (int64_t)bytes > max_device_bytes()) {
    set_error("%s: %zu bytes would exceed EF_MAX_DEVICE_BYTES", what, bytes);
    return EF_ERR_NOMEM;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("%s: device allocation of %zu bytes failed", what, bytes);
    return EF_ERR_NOMEM;
  }
  g.owned_bytes += (int64_t)bytes;
  return EF_OK;
}

static void dev_free(Graph &g, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  g.owned_bytes -= (int64_t)(bytes ? bytes : 8);
}

static ef_status ws_ensure(Graph &g, int slot, size_t bytes, const char *what) {
  DevBuf &b = g.ws[slot];
  if (b.bytes >= bytes && b.p) return EF_OK;
  if (b.p) {
    dev_free(g, b.p, b.bytes);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 256);
  ef_status s = dev_alloc(g, &b.p, want, what);
  if (s != EF_OK) return s;
  b.bytes = want;
  return EF_OK;
}

static ef_status check_device(int *dev) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    set_error("no HIP device visible");
    return EF_ERR_DEVICE;
  }
  e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_status(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, *dev);
  if (e != hipSuccess) return hip_status(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error("device %d is %s; this library is built for gfx950", *dev, prop.gcnArchName);
    return EF_ERR_DEVICE;
  }
  return EF_OK;
}

static inline bool rank_less_h(int32_t a, int32_t ka, int32_t b, int32_t kb) {
  return ka < kb || (ka == kb && a < b);
}

// Largest degree for which every cluster degree (< 3 k_max) is exact in
// FP32 and every D(s) (< 6 k_max^3) fits in int64.

}  // namespace efi

using namespace efi;

extern "C" {

const char *ef_last_error(void) { return t_err.c_str(); }

int32_t ef_version(void) { return 10000; }

ef_status ef_device_count(int32_t *count) {
  if (!count) {
    set_error("ef_device_count: null output");
    return EF_ERR_ARG;
  }
  *count = 0;
  int c = 0;
  if (hipGetDeviceCount(&c) != hipSuccess) {
    (void)hipGetLastError();
    return EF_OK;
  }
  int32_t ok = 0;
  for (int i = 0; i < c; ++i) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, i) == hipSuccess &&
        std::strncmp(prop.gcnArchName, "gfx950", 6) == 0)
      ++ok;
  }
  *count = ok;
  return EF_OK;
}

ef_status ef_validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx) {
  char msg[256] = "";
  const ef_status s = csr_validate(n, nnz, row_ptr, col_idx, msg, sizeof(msg));
  if (s != EF_OK) set_error("ef_validate_csr: %s", msg);
  return s;
}

ef_status ef_graph_free(ef_graph *h) {
  if (!h) {
    set_error("ef_graph_free: null handle");
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  if (!g.borrowed) {
    (void)hipFree(g.row_ptr);
    (void)hipFree(g.col_idx);
  }
  void *arrays[] = {g.deg, g.src, g.rev, g.rrev, g.adj2, g.adjs, g.asum, g.qa, g.nbm, g.up_ptr, g.up_col, g.trec,
                    g.up_deg, g.dn_ptr, g.dn, g.tri_zero, g.j3_seeds, g.j3_off,
                    g.tri_rec0, g.tri_recL, g.tri_list[0], g.tri_list[1], g.tri_list[2], g.tri_list[3],
                    g.tri_recB[1], g.tri_recB[2], g.fin_list,
                    g.ps_list[0], g.ps_list[1], g.ps_list[2], g.ps_list[3], g.ps_list[4],
                    g.d_counters};
  for (void *p : arrays)
    if (p) (void)hipFree(p);
  for (auto &b : g.ws)
    if (b.p) (void)hipFree(b.p);
  if (g.ev_ready)
    for (auto &e : g.ev) (void)hipEventDestroy(e);
  delete h;
  return EF_OK;
}

ef_status ef_graph_load_csr(int32_t n, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col_idx, uint32_t flags, void *hip_stream,
                            ef_graph **out) {
  return efi::graph_load(n, nnz, row_ptr, col_idx, flags, hip_stream, nullptr, 0, out);
}

}  // extern "C"

namespace efi {

ef_status graph_load(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                     uint32_t flags, void *hip_stream, const int64_t *part_off, int32_t n_parts,
                     ef_graph **out) {
  if (!out) {
    set_error("ef_graph_load_csr: null output handle");
    return EF_ERR_ARG;
  }
  *out = nullptr;
  if (n < 0 || nnz < 0 || !row_ptr || (nnz > 0 && !col_idx)) {
    set_error("ef_graph_load_csr: bad arguments (n=%d, nnz=%lld)", n, (long long)nnz);
    return EF_ERR_ARG;
  }
  if (flags & ~(EF_VALIDATE | EF_DEVICE_PTRS)) {
    set_error("ef_graph_load_csr: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  if (nnz >= (int64_t)INT32_MAX) {
    set_error("ef_graph_load_csr: nnz=%lld does not fit int32 offsets", (long long)nnz);
    return EF_ERR_OVERFLOW;
  }
  hipStream_t stream = (hipStream_t)hip_stream;
  const bool devptr = (flags & EF_DEVICE_PTRS) != 0;
  int dev = 0;
  ef_status st = EF_OK;

  // host view of the CSR (needed for validation and for sizing work lists)
  std::vector<int32_t> h_rp, h_ci;
  const int32_t *hrp = row_ptr, *hci = col_idx;
  if (devptr) {
    if ((st = check_device(&dev)) != EF_OK) return st;
    h_rp.resize((size_t)n + 1);
    hipError_t e = hipMemcpy(h_rp.data(), row_ptr, sizeof(int32_t) * ((size_t)n + 1),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_status(e, "copy row_ptr to host");
    hrp = h_rp.data();
    if (flags & EF_VALIDATE) {
      h_ci.resize((size_t)std::max<int64_t>(nnz, 1));
      if (nnz > 0) {
        e = hipMemcpy(h_ci.data(), col_idx, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_status(e, "copy col_idx to host");
      }
      hci = h_ci.data();
    }
  }
  if (flags & EF_VALIDATE) {
    st = ef_validate_csr(n, nnz, hrp, hci);
    if (st != EF_OK) return st;
  } else {
    // Without the full validation the arrays must still be safe to index
    // before any kernel reads them: offsets are checked here, neighbour ids
    // here for host input and by a device pass for device input.
    char msg[256] = "";
    st = csr_check_bounds(n, nnz, hrp, devptr ? nullptr : hci, msg, sizeof(msg));
    if (st != EF_OK) {
      set_error("ef_graph_load_csr: %s", msg);
      return st;
    }
  }
  int32_t kmax = 0;
  for (int32_t v = 0; v < n; ++v) kmax = std::max(kmax, hrp[v + 1] - hrp[v]);
  if (kmax > kMaxDegree) {
    set_error("max degree %d exceeds %d (exact cluster degrees / int64 sums)", kmax, kMaxDegree);
    return EF_ERR_OVERFLOW;
  }
  // the arrays every graph holds, against EF_MAX_DEVICE_BYTES, before the
  // device is touched (graph-dependent arrays are accounted as allocated)
  {
    const int64_t n1 = (int64_t)n + 1, m = std::max<int64_t>(nnz, 1),
                  mu = std::max<int64_t>(nnz / 2, 1), nn = std::max<int64_t>(n, 1);
    const int64_t need = (devptr ? 0 : 4 * n1 + 4 * m) + 4 * nn + (4 + 4 + 8 + 4) * m +
                         (8 + 16) * nn + 2 * 4 * n1 + (4 + 4 + 16) * mu + 256;
    if (need > max_device_bytes()) {
      set_error("ef_graph_load_csr: the graph's %lld device bytes would exceed "
                "EF_MAX_DEVICE_BYTES", (long long)need);
      return EF_ERR_NOMEM;
    }
  }
  if (!devptr && (st = check_device(&dev)) != EF_OK) return st;

  ef_graph *h = new (std::nothrow) ef_graph();
  if (!h) {
    set_error("host allocation failed");
    return EF_ERR_NOMEM;
  }
  Graph &g = h->g;
  g.dev = dev;
  g.n = n;
  g.nnz = nnz;
  g.borrowed = devptr;
  const size_t N1 = (size_t)n + 1, NNZ = (size_t)std::max<int64_t>(nnz, 1);
  const size_t NUP = (size_t)std::max<int64_t>(nnz / 2, 1);
#define ALLOC(ptr, bytes, what)                                   \
  do {                                                            \
    st = dev_alloc(g, (void **)&(ptr), (bytes), what);            \
    if (st != EF_OK) { ef_graph_free(h); return st; }             \
  } while (0)
  if (devptr) {
    g.row_ptr = const_cast<int32_t *>(row_ptr);
    g.col_idx = const_cast<int32_t *>(col_idx);
  } else {
    ALLOC(g.row_ptr, sizeof(int32_t) * N1, "row_ptr");
    ALLOC(g.col_idx, sizeof(int32_t) * NNZ, "col_idx");
    hipError_t e = hipMemcpyAsync(g.row_ptr, row_ptr, sizeof(int32_t) * N1,
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && nnz > 0)
      e = hipMemcpyAsync(g.col_idx, col_idx, sizeof(int32_t) * (size_t)nnz,
                         hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
      ef_graph_free(h);
      return hip_status(e, "copy CSR to device");
    }
  }
  ALLOC(g.deg, sizeof(int32_t) * std::max<size_t>(n, 1), "deg");
  ALLOC(g.src, sizeof(int32_t) * NNZ, "src");
  ALLOC(g.rev, sizeof(int32_t) * NNZ, "rev");
  ALLOC(g.rrev, sizeof(int32_t) * NNZ, "reverse sum index");
  ALLOC(g.adj2, sizeof(int2) * NNZ, "adj2");
  ALLOC(g.asum, sizeof(int64_t) * std::max<size_t>(n, 1), "asum");
  ALLOC(g.qa, sizeof(longlong2) * std::max<size_t>(n, 1), "qa");
  ALLOC(g.nbm, sizeof(NbrMoments) * std::max<size_t>(n, 1), "neighbour degree moments");
  ALLOC(g.up_ptr, sizeof(int32_t) * N1, "up_ptr");
  ALLOC(g.up_col, sizeof(int32_t) * NUP, "up_col");
  ALLOC(g.up_deg, sizeof(int32_t) * NUP, "up_deg");
  ALLOC(g.trec, sizeof(int32_t) * NNZ, "triangle record index");
  ALLOC(g.dn_ptr, sizeof(int32_t) * N1, "dn_ptr");
  ALLOC(g.dn, sizeof(int4) * NUP, "triangle segments");
  ALLOC(g.d_counters, sizeof(int32_t) * 64, "counters");
  if (devptr && !(flags & EF_VALIDATE) && nnz > 0) {
    // neighbour ids of borrowed device arrays: in range before any kernel
    // indexes with them
    int32_t bad = 0;
    hipError_t e = launch_check_cols(g.col_idx, nnz, n, g.d_counters, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&bad, g.d_counters, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      ef_graph_free(h);
      return hip_status(e, "check neighbour ids");
    }
    if (bad) {
      ef_graph_free(h);
      set_error("ef_graph_load_csr: a neighbour id is outside [0, %d)", n);
      return EF_ERR_RANGE;
    }
  }
  // tail entries walked at each node by the triangle pass (binning)
  std::vector<int64_t> h_work((size_t)n);
  {
    int32_t *tmp = nullptr;
    int64_t *work = nullptr;
    const size_t tmp_bytes = sizeof(int32_t) * (size_t)graph_prep_tmp_len((int64_t)NNZ);
    const size_t work_bytes = sizeof(int64_t) * std::max<size_t>(n, 1);
    ALLOC(tmp, tmp_bytes, "preprocessing scratch");
    st = dev_alloc(g, (void **)&work, work_bytes, "preprocessing scratch");
    if (st != EF_OK) {
      dev_free(g, tmp, tmp_bytes);
      ef_graph_free(h);
      return st;
    }
    bool not_symmetric = false;
    hipError_t e = launch_graph_prep(g, tmp, work, not_symmetric, stream);
    // the reverse-sum index starts as rev; big centres' rows remap it below
    if (e == hipSuccess)
      e = hipMemcpyAsync(g.rrev, g.rev, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice,
                         stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess && not_symmetric) {
      dev_free(g, work, work_bytes);
      dev_free(g, tmp, tmp_bytes);
      ef_graph_free(h);
      set_error("the CSR is not simple and symmetric (load with EF_VALIDATE for details)");
      return EF_ERR_NOT_SYMMETRIC;
    }
    if (e == hipSuccess) e = graph_zero_count(g, tmp, g.n_tri_zero);
    if (e == hipSuccess) {
      st = dev_alloc(g, (void **)&g.tri_zero,
                     sizeof(int32_t) * (size_t)std::max<int64_t>(g.n_tri_zero, 1), "zero slots");
      if (st == EF_OK) {
        e = launch_zero_list(g, tmp, stream);
        if (e == hipSuccess && n > 0)
          e = hipMemcpyAsync(h_work.data(), work, sizeof(int64_t) * (size_t)n,
                             hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
      }
    }
    dev_free(g, work, work_bytes);
    dev_free(g, tmp, tmp_bytes);
    if (st != EF_OK) {
      ef_graph_free(h);
      return st;
    }
    if (e != hipSuccess) {
      ef_graph_free(h);
      return hip_status(e, "graph preprocessing");
    }
  }
  std::vector<int32_t> h_dn_ptr(N1);
  {
    hipError_t e = hipMemcpy(h_dn_ptr.data(), g.dn_ptr, sizeof(int32_t) * N1,
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      ef_graph_free(h);
      return hip_status(e, "copy dn_ptr to host");
    }
  }
  // host copies: degrees and |up(u)|
  g.h_deg.resize((size_t)n);
  for (int32_t v = 0; v < n; ++v) g.h_deg[v] = hrp[v + 1] - hrp[v];
  std::vector<int32_t> h_up_ptr(N1);
  {
    hipError_t e = hipMemcpy(h_up_ptr.data(), g.up_ptr, sizeof(int32_t) * N1,
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      ef_graph_free(h);
      return hip_status(e, "copy up_ptr to host");
    }
  }
  g.h_up_len.resize((size_t)n);
  ef_graph_info &inf = g.info;
  inf.n = n;
  inf.nnz = nnz;
  inf.max_degree = kmax;
  inf.up_arcs = nnz / 2;
  // degree-ordered rows of the mid and big centres (the tile pair loops,
  // which store their per-arc sums by sorted position)
  {
    std::vector<int32_t> hb;
    for (int32_t v = 0; v < n; ++v)
      if (g.h_deg[v] > kSmallMax) hb.push_back(v);
    if (!hb.empty()) {
      ALLOC(g.adjs, sizeof(int2) * NNZ, "degree-ordered rows");
      const int32_t nbig = (int32_t)hb.size();
      const size_t sb = sizeof(int32_t) * 4 * NNZ, gb = sizeof(int32_t) * 2 * (size_t)nbig,
                   bb = sizeof(int32_t) * (size_t)nbig;
      int32_t *scratch = nullptr, *seg = nullptr, *d_big = nullptr;
      void *temp = nullptr;
      size_t temp_bytes = 0;
      st = dev_alloc(g, (void **)&scratch, sb, "sort scratch");
      if (st == EF_OK) st = dev_alloc(g, (void **)&seg, gb, "sort segments");
      if (st == EF_OK) st = dev_alloc(g, (void **)&d_big, bb, "big centres");
      hipError_t e = hipSuccess;
      if (st == EF_OK) {
        e = hipMemcpyAsync(d_big, hb.data(), bb, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
          e = launch_big_sort(g, d_big, nbig, scratch, seg, nullptr, temp_bytes, stream);
        if (e == hipSuccess) st = dev_alloc(g, &temp, temp_bytes, "sort scratch");
        if (e == hipSuccess && st == EF_OK)
          e = launch_big_sort(g, d_big, nbig, scratch, seg, temp, temp_bytes, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
      }
      dev_free(g, temp, temp_bytes);
      dev_free(g, d_big, bb);
      dev_free(g, seg, gb);
      dev_free(g, scratch, sb);
      if (st == EF_OK && e != hipSuccess) st = hip_status(e, "degree-ordered rows");
      if (st != EF_OK) {
        ef_graph_free(h);
        return st;
      }
    }
  }
  std::vector<int32_t> tri[4], fin, fin_group;
  std::vector<int4> recL;
  for (int32_t v = 0; v < n; ++v) {
    const int64_t k = g.h_deg[v];
    const int32_t up = h_up_ptr[v + 1] - h_up_ptr[v];
    g.h_up_len[v] = up;
    inf.clusters += k * (k - 1) / 2;
    inf.sum_sq_degree += k * k;
    inf.wedge_checks += h_work[v];
    if (k >= 2 && k <= kSmallMax) {
      g.all_small++;
      g.all_small_deg[k]++;
      g.all_pairs_small += k * (k - 1) / 2;
    } else if (k > kSmallMax && k <= kSuper) {
      g.all_mid++;
      g.all_midc[mid_class((int32_t)k)]++;
      g.all_pairs_mid += k * (k - 1) / 2;
    } else if (k > kSuper) {
      const int64_t ns = (k + kSuper - 1) / kSuper;
      g.all_big++;
      g.all_tiles += ns * (ns + 1) / 2;
      g.all_pairs_big += k * (k - 1) / 2;
      g.all_sblocks += ns;
    }
    const int32_t nd = h_dn_ptr[v + 1] - h_dn_ptr[v];
    if (nd > 0 && up <= kTriLaneM && h_work[v] <= kTriLaneWork && nd <= kTriLaneSegs) {
      recL.push_back(make_int4(v, h_up_ptr[v], h_dn_ptr[v],
                               up | (nd << 8) | ((int32_t)h_work[v] << 16)));
    } else if (nd > 0) {
      const int bin = (up <= kTriBin0 && h_work[v] <= kTriWaveWork && nd <= kTriWaveSegs) ? 0
                      : up <= kTriBin1                                                  ? 1
                      : up <= kTriBin2                                                  ? 2
                                                                                        : 3;
      tri[bin].push_back(v);
    }
    if (k > kFinGroupMax) fin.push_back(v);
    else if (k > kFinLaneMax) fin_group.push_back(v);
  }
  // graph by graph when the nodes are a union of parts (a batch), then
  // longest walks first
  std::vector<int32_t> part;
  if (part_off && n_parts > 0) {
    part.resize((size_t)n);
    for (int32_t q = 0; q < n_parts; ++q)
      for (int64_t v = part_off[q]; v < part_off[q + 1]; ++v) part[(size_t)v] = q;
  }
  auto part_of = [&](int32_t v) { return part.empty() ? 0 : part[(size_t)v]; };
  auto by_work = [&](int32_t a, int32_t b) {
    if (part_of(a) != part_of(b)) return part_of(a) < part_of(b);
    return h_work[a] != h_work[b] ? h_work[a] > h_work[b] : a < b;
  };
  for (int bin = 0; bin < 4; ++bin) {
    std::sort(tri[bin].begin(), tri[bin].end(), by_work);
    g.n_tri[bin] = (int64_t)tri[bin].size();
    if (bin > 0)
      ALLOC(g.tri_list[bin], sizeof(int32_t) * std::max<size_t>(tri[bin].size(), 1),
            "triangle list");
  }
  std::vector<int4> rec0(tri[0].size());
  for (size_t i = 0; i < tri[0].size(); ++i) {
    const int32_t v = tri[0][i];
    const int32_t m = h_up_ptr[v + 1] - h_up_ptr[v], nd = h_dn_ptr[v + 1] - h_dn_ptr[v];
    rec0[i] = make_int4(v, h_up_ptr[v], h_dn_ptr[v], m | (nd << 16));
  }
  ALLOC(g.tri_rec0, sizeof(int4) * std::max<size_t>(rec0.size(), 1), "triangle records");
  // workgroup bins: |up(w)| <= kTriBin2 < 2^12, segments <= degree < 2^20
  static_assert(kTriBin2 < (1 << 12) && kMaxDegree < (1 << 20), "workgroup-bin record packing");
  std::vector<int4> recB[3];
  for (int bin = 1; bin <= 2; ++bin) {
    recB[bin].resize(tri[bin].size());
    for (size_t i = 0; i < tri[bin].size(); ++i) {
      const int32_t v = tri[bin][i];
      const int32_t m = h_up_ptr[v + 1] - h_up_ptr[v], nd = h_dn_ptr[v + 1] - h_dn_ptr[v];
      recB[bin][i] = make_int4(v, h_up_ptr[v], h_dn_ptr[v], m | (nd << 12));
    }
    ALLOC(g.tri_recB[bin], sizeof(int4) * std::max<size_t>(recB[bin].size(), 1),
          "triangle records");
  }
  g.n_tri_lane = (int64_t)recL.size();
  ALLOC(g.tri_recL, sizeof(int4) * std::max<size_t>(recL.size(), 1), "triangle lane records");
  // tiers by degree (descending), each graph by graph
  auto fin_tier = [&](int32_t v) {
    return g.h_deg[v] > kFinBlockMin ? 0 : g.h_deg[v] > kFinHalfMax ? 1 : 2;
  };
  std::sort(fin.begin(), fin.end(), [&](int32_t a, int32_t b) {
    if (fin_tier(a) != fin_tier(b)) return fin_tier(a) < fin_tier(b);
    if (part_of(a) != part_of(b)) return part_of(a) < part_of(b);
    return g.h_deg[a] != g.h_deg[b] ? g.h_deg[a] > g.h_deg[b] : a < b;
  });
  g.n_fin = (int64_t)fin.size();
  for (int32_t v : fin)
    if (g.h_deg[v] > kFinBlockMin) g.n_fin_hub++;
    else if (g.h_deg[v] <= kFinHalfMax) g.n_fin_half++;
  g.n_fin_group = (int64_t)fin_group.size();
  fin.insert(fin.end(), fin_group.begin(), fin_group.end());
  if (!part.empty()) {
    // node ids of the lists, for schedules that split them by graph
    g.h_fin = fin;
    for (int bin = 0; bin < 4; ++bin) g.h_tri[bin] = tri[bin];
    g.h_tri_lane.resize(recL.size());
    for (size_t i = 0; i < recL.size(); ++i) g.h_tri_lane[i] = recL[i].x;
  }
  ALLOC(g.fin_list, sizeof(int32_t) * std::max<size_t>(fin.size(), 1), "finalize list");
#undef ALLOC
  hipError_t e = hipSuccess;
  for (int bin = 1; bin < 4 && e == hipSuccess; ++bin)
    if (!tri[bin].empty())
      e = hipMemcpy(g.tri_list[bin], tri[bin].data(), sizeof(int32_t) * tri[bin].size(),
                    hipMemcpyHostToDevice);
  if (e == hipSuccess && !rec0.empty())
    e = hipMemcpy(g.tri_rec0, rec0.data(), sizeof(int4) * rec0.size(), hipMemcpyHostToDevice);
  for (int bin = 1; bin <= 2 && e == hipSuccess; ++bin)
    if (!recB[bin].empty())
      e = hipMemcpy(g.tri_recB[bin], recB[bin].data(), sizeof(int4) * recB[bin].size(),
                    hipMemcpyHostToDevice);
  if (e == hipSuccess && !recL.empty())
    e = hipMemcpy(g.tri_recL, recL.data(), sizeof(int4) * recL.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !fin.empty())
    e = hipMemcpy(g.fin_list, fin.data(), sizeof(int32_t) * fin.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    ef_graph_free(h);
    return hip_status(e, "upload node lists");
  }
  *out = h;
  return EF_OK;
}

}  // namespace efi

extern "C" {

ef_status ef_graph_from_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                              void *hip_stream, ef_graph **out) {
  if (!out || n < 0 || m < 0 || (m > 0 && (!src || !dst))) {
    set_error("ef_graph_from_edges: bad arguments");
    return EF_ERR_ARG;
  }
  std::vector<int64_t> cnt((size_t)n + 1, 0);
  for (int64_t i = 0; i < m; ++i) {
    const int32_t u = src[i], v = dst[i];
    if (u < 0 || u >= n || v < 0 || v >= n) {
      set_error("edge %lld: endpoint out of range [0, %d)", (long long)i, n);
      return EF_ERR_RANGE;
    }
    if (u == v) continue;
    cnt[u + 1]++;
    cnt[v + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  if (cnt[n] >= (int64_t)INT32_MAX) {
    set_error("ef_graph_from_edges: too many arcs");
    return EF_ERR_OVERFLOW;
  }
  std::vector<int32_t> col((size_t)cnt[n]);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < m; ++i) {
    const int32_t u = src[i], v = dst[i];
    if (u == v) continue;
    col[pos[u]++] = v;
    col[pos[v]++] = u;
  }
  std::vector<int32_t> rp((size_t)n + 1, 0);
  int64_t w = 0;
  for (int32_t v = 0; v < n; ++v) {
    auto b = col.begin() + cnt[v], e = col.begin() + cnt[v + 1];
    std::sort(b, e);
    auto last = std::unique(b, e);
    for (auto it = b; it != last; ++it) col[w++] = *it;
    rp[v + 1] = (int32_t)w;
  }
  return ef_graph_load_csr(n, w, rp.data(), col.data(), 0, hip_stream, out);
}

ef_status ef_graph_info_get(const ef_graph *h, ef_graph_info *out) {
  if (!h || !out) {
    set_error("ef_graph_info_get: null argument");
    return EF_ERR_ARG;
  }
  *out = h->g.info;
  return EF_OK;
}

ef_status ef_stats(const ef_graph *h, ef_run_stats *out) {
  if (!h || !out) {
    set_error("ef_stats: null argument");
    return EF_ERR_ARG;
  }
  *out = h->g.stats;
  return EF_OK;
}

}  // extern "C"

namespace efi {

// workspace slots
enum {
  WS_R = 0, WS_REC, WS_Y, WS_Z, WS_ZT, WS_FLAG, WS_BINS, WS_OUT, WS_BITMAP,
  WS_SEEDS, WS_UOUT, WS_TOPK, WS_SURR, WS_J3, WS_J3P, WS_J3L
};

// scratch for other translation units (kept in the handle, grow-only)
ef_status graph_scratch(Graph &g, size_t bytes, void **out) {
  ef_status s = ws_ensure(g, WS_SURR, bytes, "scratch");
  *out = s == EF_OK ? g.ws[WS_SURR].p : nullptr;
  return s;
}

static void host_bins(const Graph &g, const int32_t *centres, int64_t count, Bins &b) {
  b.n_small = b.n_mid = b.n_big = b.n_tiles = 0;
  b.pairs_small = b.pairs_mid = b.pairs_big = 0;
  b.n_sblocks = 0;
  for (auto &c : b.n_smallb) c = 0;
  for (auto &c : b.n_midc) c = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t k = g.h_deg[centres ? centres[i] : i];
    if (k < 2) continue;
    if (k <= kSmallMax) {
      b.n_small++;
      b.n_smallb[small_bin((int32_t)k, b.thr)]++;
      b.pairs_small += k * (k - 1) / 2;
    } else if (k <= kSuper) {
      b.n_mid++;
      b.n_midc[mid_class((int32_t)k)]++;
      b.pairs_mid += k * (k - 1) / 2;
    } else {
      const int64_t ns = (k + kSuper - 1) / kSuper;
      b.n_big++;
      b.n_tiles += ns * (ns + 1) / 2;
      b.pairs_big += k * (k - 1) / 2;
      b.n_sblocks += ns;
    }
  }
}

static ef_status alloc_bins(Graph &g, Bins &b) {
  const size_t bytes = sizeof(int32_t) * (size_t)(b.n_small + 2 * b.n_mid + 16) + 8 * 256 +
                       sizeof(BigCentre) * (size_t)(b.n_big + 1) +
                       sizeof(int32_t) * (size_t)(b.n_big + 1) +
                       sizeof(TileItem) * (size_t)(b.n_tiles + 1) +
                       sizeof(int2) * (size_t)(b.n_sblocks + 1) + 4096;
  ef_status s = ws_ensure(g, WS_BINS, bytes, "work lists");
  if (s != EF_OK) return s;
  char *p = (char *)g.ws[WS_BINS].p;
  auto take = [&](size_t n) {
    char *r = p;
    p += (n + 255) & ~(size_t)255;
    return r;
  };
  b.counters = (int32_t *)take(sizeof(int32_t) * 16);
  for (int i = 0; i < 4; ++i)
    b.small[i] = (int32_t *)take(sizeof(int32_t) * (size_t)(b.n_smallb[i] + 1));
  b.mid = (int32_t *)take(sizeof(int32_t) * (size_t)(b.n_mid + 1));
  for (int c = 0; c < 3; ++c)
    b.midc[c] = (int32_t *)take(sizeof(int32_t) * (size_t)(b.n_midc[c] + 1));
  b.big = (BigCentre *)take(sizeof(BigCentre) * (size_t)(b.n_big + 1));
  b.agg_done = (int32_t *)take(sizeof(int32_t) * (size_t)(b.n_big + 1));
  b.tiles = (TileItem *)take(sizeof(TileItem) * (size_t)(b.n_tiles + 1));
  b.sblocks = (int2 *)take(sizeof(int2) * (size_t)(b.n_sblocks + 1));
  return EF_OK;
}

struct Prof {
  Graph &g;
  bool on;
  hipStream_t st;
  int used = 0;
  int idx[16];
  Prof(Graph &gg, bool o, hipStream_t s) : g(gg), on(o), st(s) {}
  ef_status init() {
    if (!on || g.ev_ready) return EF_OK;
    for (auto &e : g.ev) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return hip_status(r, "hipEventCreate");
    }
    g.ev_ready = true;
    return EF_OK;
  }
  hipEvent_t ev(int i) { return on ? g.ev[i] : nullptr; }
  void mark(int i) {
    if (on) (void)hipEventRecord(g.ev[i], st);
  }
  double ms(int a, int b) {
    float t = 0.f;
    if (!on) return 0.0;
    if (hipEventElapsedTime(&t, g.ev[a], g.ev[b]) != hipSuccess) {
      (void)hipGetLastError();
      return 0.0;
    }
    return (double)t;
  }
};

}  // namespace efi

extern "C" ef_status ef_compute(ef_graph *h, ef_algo algo, ef_prec prec, const int32_t *seeds,
                                int32_t n_seeds, double *ef, int64_t *D, int64_t *N,
                                uint32_t flags, void *hip_stream) {
  if (!h || !ef) {
    set_error("ef_compute: null handle or output");
    return EF_ERR_ARG;
  }
  if ((algo != EF_ALGO_CLUSTER && algo != EF_ALGO_PER_SEED && algo != EF_ALGO_CLUSTER_AGG) ||
      (prec != EF_PREC_FP64 && prec != EF_PREC_FP32C)) {
    set_error("ef_compute: bad algorithm or precision");
    return EF_ERR_ARG;
  }
  if (flags & ~(EF_OUT_DEVICE | EF_PROFILE | kInternalNoReadback)) {
    set_error("ef_compute: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  if (seeds && n_seeds < 0) {
    set_error("ef_compute: negative n_seeds");
    return EF_ERR_ARG;
  }
  if (seeds && n_seeds == 0) return EF_OK;
  if (seeds) {
    for (int32_t i = 0; i < n_seeds; ++i)
      if (seeds[i] < 0 || seeds[i] >= g.n) {
        set_error("ef_compute: seed %d at position %d out of range [0, %d)", seeds[i], i, g.n);
        return EF_ERR_RANGE;
      }
  }
  if (!seeds && g.n == 0) return EF_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const bool out_dev = (flags & EF_OUT_DEVICE) != 0;
  Prof prof(g, (flags & EF_PROFILE) != 0, st);
  ef_status s = prof.init();
  if (s != EF_OK) return s;
  g.stats = ef_run_stats{};
  const size_t tsz = prec == EF_PREC_FP64 ? sizeof(double) : sizeof(float2);
  const int64_t nnz = std::max<int64_t>(g.nnz, 1), nup = std::max<int64_t>(g.nnz / 2, 1);

  // seeds: unique sorted list + inverse map
  const bool all = seeds == nullptr;
  std::vector<int32_t> useeds, inv;
  int32_t n_out = all ? g.n : n_seeds;
  if (!all) {
    useeds.assign(seeds, seeds + n_seeds);
    std::sort(useeds.begin(), useeds.end());
    useeds.erase(std::unique(useeds.begin(), useeds.end()), useeds.end());
    inv.resize((size_t)n_seeds);
    for (int32_t i = 0; i < n_seeds; ++i)
      inv[i] = (int32_t)(std::lower_bound(useeds.begin(), useeds.end(), seeds[i]) - useeds.begin());
  }
  const bool per_seed = !all || algo == EF_ALGO_PER_SEED;
  const int32_t n_work = all ? g.n : (int32_t)useeds.size();

  // work lists of the pair loop
  Bins b;
  if (all) {
    b.thr = g.thr;
    b.n_small = g.all_small;
    for (int k = 2; k <= kSmallMax; ++k) b.n_smallb[small_bin(k, b.thr)] += g.all_small_deg[k];
    b.n_mid = g.all_mid;
    for (int c = 0; c < 3; ++c) b.n_midc[c] = g.all_midc[c];
    b.n_big = g.all_big;
    b.n_tiles = g.all_tiles;
    b.pairs_small = g.all_pairs_small;
    b.pairs_mid = g.all_pairs_mid;
    b.pairs_big = g.all_pairs_big;
    b.n_sblocks = g.all_sblocks;
  } else {
    b.thr = g.thr;
    host_bins(g, useeds.data(), (int64_t)useeds.size(), b);
  }
  if ((s = alloc_bins(g, b)) != EF_OK) return s;
  // per-arc sums: one float (FP32C) or double each
  const size_t asz = prec == EF_PREC_FP64 ? sizeof(double) : sizeof(float);
  if ((s = ws_ensure(g, WS_R, asz * (size_t)nnz, "arc sums")) != EF_OK) return s;
  // super-tile record entries: one float (FP32C) or double each
  const size_t rsz = prec == EF_PREC_FP64 ? sizeof(double) : sizeof(float);
  if ((s = ws_ensure(g, WS_REC, rsz * (size_t)kRecEntries * (size_t)std::max<int64_t>(b.n_tiles, 1),
                     "super-tile records")) != EF_OK)
    return s;
  if ((s = ws_ensure(g, WS_FLAG, (sizeof(int32_t) + 1) * (size_t)std::max<int32_t>(n_work, 1),
                     "flag list")) != EF_OK)
    return s;
  // outputs of the unique work list: straight into the caller's device arrays
  // when possible, else into staging
  double *ef_w = nullptr;
  int64_t *D_w = nullptr, *N_w = nullptr;
  const size_t out_bytes = (sizeof(double) + 2 * sizeof(int64_t)) * (size_t)std::max(n_work, 1);
  if ((s = ws_ensure(g, WS_UOUT, out_bytes, "output staging")) != EF_OK) return s;
  {
    char *p = (char *)g.ws[WS_UOUT].p;
    ef_w = (double *)p;
    D_w = (int64_t *)(p + sizeof(double) * (size_t)std::max(n_work, 1));
    N_w = D_w + std::max(n_work, 1);
    if (all && out_dev) {
      ef_w = ef;
      if (D) D_w = D;
      if (N) N_w = N;
    }
  }
  int32_t *cnt = g.d_counters;  // [0] flagged, [1] fp64-finalised
  hipError_t e = launch_zero_i32(cnt, 4, st);
  if (e != hipSuccess) return hip_status(e, "clear counters");
  int32_t *flagged = (int32_t *)g.ws[WS_FLAG].p;
  uint8_t *flag_bytes = (uint8_t *)(flagged + std::max<int32_t>(n_work, 1));

  // device seed arrays: the unique work list (all nodes: none, position =
  // node id), the inverse map, and output positions by seed degree bin
  int32_t *d_useeds = nullptr, *d_inv = nullptr;
  const int32_t *ps_lists[kSeedBins] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t ps_counts[kSeedBins] = {0, 0, 0, 0, 0};
  if (per_seed && g.h_asum.empty() && g.n > 0) {
    g.h_asum.resize((size_t)g.n);
    e = hipMemcpy(g.h_asum.data(), g.asum, sizeof(int64_t) * (size_t)g.n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      g.h_asum.clear();
      return hip_status(e, "copy neighbour-degree sums");
    }
  }
  auto seed_bin = [&](int32_t v) {
    const int32_t k = g.h_deg[v];
    if (k <= kSeedBin0 && g.h_asum[v] <= kSeedWaveWork) return 0;
    return k <= kSeedBin1 ? 1 : k <= kSeedBin2 ? 2 : k <= kSeedBin3 ? 3 : 4;
  };
  // largest 2-hop work first
  auto by_work = [&](int32_t a, int32_t c) {
    const int64_t wa = g.h_asum[a], wc = g.h_asum[c];
    return wa != wc ? wa > wc : a < c;
  };
  if (per_seed && all) {
    if (!g.ps_ready) {
      std::vector<int32_t> lst[kSeedBins];
      for (int32_t v = 0; v < g.n; ++v) lst[seed_bin(v)].push_back(v);
      for (int bin = 0; bin < kSeedBins; ++bin) {
        std::sort(lst[bin].begin(), lst[bin].end(), by_work);
        g.n_ps[bin] = (int64_t)lst[bin].size();
        if ((s = dev_alloc(g, (void **)&g.ps_list[bin],
                           sizeof(int32_t) * std::max<size_t>(lst[bin].size(), 1),
                           "seed lists")) != EF_OK)
          return s;
        if (!lst[bin].empty()) {
          e = hipMemcpy(g.ps_list[bin], lst[bin].data(), sizeof(int32_t) * lst[bin].size(),
                        hipMemcpyHostToDevice);
          if (e != hipSuccess) return hip_status(e, "upload seed lists");
        }
      }
      g.ps_ready = true;
    }
    for (int bin = 0; bin < kSeedBins; ++bin) {
      ps_lists[bin] = g.ps_list[bin];
      ps_counts[bin] = g.n_ps[bin];
    }
  } else if (per_seed) {
    std::vector<int32_t> lst[kSeedBins];
    std::vector<int32_t> order(useeds.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int32_t a, int32_t c) { return by_work(useeds[a], useeds[c]); });
    for (int32_t i : order) lst[seed_bin(useeds[i])].push_back(i);
    const size_t cnt_all = useeds.size() * 2 + inv.size() + 4;
    if ((s = ws_ensure(g, WS_SEEDS, sizeof(int32_t) * cnt_all, "seed lists")) != EF_OK) return s;
    d_useeds = (int32_t *)g.ws[WS_SEEDS].p;
    int32_t *p = d_useeds + useeds.size();
    e = hipMemcpyAsync(d_useeds, useeds.data(), sizeof(int32_t) * useeds.size(),
                       hipMemcpyHostToDevice, st);
    for (int bin = 0; bin < kSeedBins; ++bin) {
      ps_lists[bin] = p;
      ps_counts[bin] = (int64_t)lst[bin].size();
      if (e == hipSuccess && !lst[bin].empty())
        e = hipMemcpyAsync(p, lst[bin].data(), sizeof(int32_t) * lst[bin].size(),
                           hipMemcpyHostToDevice, st);
      p += lst[bin].size();
    }
    d_inv = p;
    if (e == hipSuccess && !inv.empty())
      e = hipMemcpyAsync(d_inv, inv.data(), sizeof(int32_t) * inv.size(), hipMemcpyHostToDevice,
                         st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // host vectors go out of scope
    if (e != hipSuccess) return hip_status(e, "upload seeds");
  }
  if (per_seed && ps_counts[kSeedBins - 1] > 0) {
    const size_t words = ((size_t)g.n + 31) / 32;
    const size_t need = sizeof(uint32_t) * words * (size_t)ps_counts[kSeedBins - 1];
    const bool fresh = g.ws[WS_BITMAP].bytes < need;
    if ((s = ws_ensure(g, WS_BITMAP, need, "membership bitmaps")) != EF_OK) return s;
    if (fresh) {
      e = hipMemsetAsync(g.ws[WS_BITMAP].p, 0, g.ws[WS_BITMAP].bytes, st);
      if (e != hipSuccess) return hip_status(e, "clear bitmaps");
    }
  }

  // whole-graph calls bin every node with the graph's thresholds: their
  // lists are kept and reused (not while the stream is being captured, so
  // that a captured graph bins by itself)
  const int32_t *centres = per_seed ? d_useeds : nullptr;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) {
    (void)hipGetLastError();
    cap = hipStreamCaptureStatusActive;
  }
  const bool whole = centres == nullptr && cap == hipStreamCaptureStatusNone;
  const bool reuse = whole && g.bins_kept && g.bins_buf == g.ws[WS_BINS].p &&
                     g.bins_thr.t8 == b.thr.t8 && g.bins_thr.t16 == b.thr.t16 &&
                     g.bins_thr.t32 == b.thr.t32;
  prof.mark(0);
  if (!reuse) {
    e = launch_bin_centres(g, centres, n_work, b, st);
    if (e != hipSuccess) return hip_status(e, "binning");
  }
  g.bins_kept = whole;
  g.bins_thr = b.thr;
  g.bins_buf = g.ws[WS_BINS].p;
  prof.mark(1);
  e = launch_pairs(g, prec, b, g.ws[WS_R].p, g.ws[WS_REC].p, st, prof.ev(2), prof.ev(3),
                   prof.ev(4), algo == EF_ALGO_CLUSTER_AGG ? b.agg_done : nullptr);
  if (e != hipSuccess) return hip_status(e, "pair loop");
  prof.mark(5);
  if (!per_seed) {
    if ((s = ws_ensure(g, WS_Y, sizeof(TriSlot) * 2 * (size_t)nup, "triangle slots")) != EF_OK)
      return s;
    if ((s = ws_ensure(g, WS_Z, tsz * (size_t)std::max(g.n, 1), "triangle node sums")) != EF_OK) return s;
    if ((s = ws_ensure(g, WS_ZT, sizeof(int64_t) * (size_t)std::max(g.n, 1), "triangle node counts")) != EF_OK)
      return s;
    e = launch_triangles(g, prec, (TriSlot *)g.ws[WS_Y].p, g.ws[WS_Z].p,
                         (int64_t *)g.ws[WS_ZT].p, st);
    if (e != hipSuccess) return hip_status(e, "triangle pass");
    prof.mark(6);
    e = launch_finalize_cluster(g, prec, g.ws[WS_R].p, (const TriSlot *)g.ws[WS_Y].p,
                                g.ws[WS_Z].p, (int64_t *)g.ws[WS_ZT].p, ef_w, D_w, N_w,
                                flag_bytes, st);
    if (e == hipSuccess) e = launch_flag_compact(flag_bytes, n_work, flagged, cnt, st);
    if (e != hipSuccess) return hip_status(e, "finalize");
    prof.mark(7);
  } else {
    e = launch_per_seed(g, prec, d_useeds, ps_lists, ps_counts, g.ws[WS_R].p,
                        (uint32_t *)g.ws[WS_BITMAP].p, ef_w, D_w, N_w, flag_bytes, st,
                        prof.ev(6));
    if (e == hipSuccess) e = launch_flag_compact(flag_bytes, n_work, flagged, cnt, st);
    if (e != hipSuccess) return hip_status(e, "per-seed stream");
    prof.mark(7);
  }
  if (prec == EF_PREC_FP32C) {
    e = launch_pass2(g, per_seed ? d_useeds : nullptr, flagged, cnt, n_work, ef_w, D_w, st);
    if (e != hipSuccess) return hip_status(e, "pass 2");
  }
  prof.mark(8);

  // deliver outputs
  if (!all) {
    if (out_dev) {
      e = launch_gather_outputs(d_inv, n_seeds, ef_w, D_w, N_w, ef, D, N, st);
      if (e != hipSuccess) return hip_status(e, "scatter outputs");
    } else {
      std::vector<double> hef((size_t)n_work);
      std::vector<int64_t> hD((size_t)n_work), hN((size_t)n_work);
      e = hipMemcpyAsync(hef.data(), ef_w, sizeof(double) * n_work, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hD.data(), D_w, sizeof(int64_t) * n_work, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hN.data(), N_w, sizeof(int64_t) * n_work, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_status(e, "copy outputs");
      for (int32_t i = 0; i < n_seeds; ++i) {
        ef[i] = hef[inv[i]];
        if (D) D[i] = hD[inv[i]];
        if (N) N[i] = hN[inv[i]];
      }
    }
  } else if (!out_dev) {
    e = hipMemcpyAsync(ef, ef_w, sizeof(double) * (size_t)n_out, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && D)
      e = hipMemcpyAsync(D, D_w, sizeof(int64_t) * (size_t)n_out, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && N)
      e = hipMemcpyAsync(N, N_w, sizeof(int64_t) * (size_t)n_out, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e, "copy outputs");
  }
  g.stats.pair_tiles = b.n_tiles;
  g.stats.pairs_small = b.pairs_small;
  g.stats.pairs_mid = b.pairs_mid;
  g.stats.pairs_big = b.pairs_big;
  g.stats.seeds = n_work;
  if ((prof.on || !out_dev) && !(flags & kInternalNoReadback)) {
    int32_t hc[2] = {0, 0};
    e = hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e, "read counters");
    g.stats.promoted = hc[0];
    g.stats.fp64_finalized = hc[1];
  }
  if (prof.on) {
    g.stats.t_bin_ms = prof.ms(0, 1);
    g.stats.t_pairs_small_ms = prof.ms(1, 2);
    g.stats.t_pairs_mid_ms = prof.ms(2, 3);
    g.stats.t_pairs_big_ms = prof.ms(3, 4);
    g.stats.t_pairs_ms = prof.ms(1, 4);
    g.stats.t_reduce_ms = prof.ms(4, 5);
    if (!per_seed) {
      g.stats.t_triangles_ms = prof.ms(5, 6);
      g.stats.t_finalize_ms = prof.ms(6, 7);
    } else {
      g.stats.t_stream_ms = prof.ms(5, 7);
    }
    g.stats.t_pass2_ms = prof.ms(7, 8);
    g.stats.t_total_ms = prof.ms(0, 8);
  }
  return EF_OK;
}

extern "C" ef_status ef_compute_j3(ef_graph *h, ef_prec prec, const int32_t *seeds,
                                   int32_t n_seeds, double *ef, int64_t *D, int64_t *N,
                                   uint32_t flags, void *hip_stream) {
  if (!h || !ef) {
    set_error("ef_compute_j3: null handle or output");
    return EF_ERR_ARG;
  }
  if (prec != EF_PREC_FP64 && prec != EF_PREC_FP32C) {
    set_error("ef_compute_j3: bad precision");
    return EF_ERR_ARG;
  }
  if (flags & ~(EF_OUT_DEVICE | EF_PROFILE)) {
    set_error("ef_compute_j3: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  if (seeds && n_seeds < 0) {
    set_error("ef_compute_j3: negative n_seeds");
    return EF_ERR_ARG;
  }
  if (seeds && n_seeds == 0) return EF_OK;
  if (seeds)
    for (int32_t i = 0; i < n_seeds; ++i)
      if (seeds[i] < 0 || seeds[i] >= g.n) {
        set_error("ef_compute_j3: seed %d at position %d out of range [0, %d)", seeds[i], i,
                  g.n);
        return EF_ERR_RANGE;
      }
  if (!seeds && g.n == 0) return EF_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const bool out_dev = (flags & EF_OUT_DEVICE) != 0;
  Prof prof(g, (flags & EF_PROFILE) != 0, st);
  ef_status s = prof.init();
  if (s != EF_OK) return s;
  g.stats = ef_run_stats{};
  hipError_t e = hipSuccess;

  // host copies of the per-node sums (work estimates and the int64 bound)
  if (g.h_asum.empty() && g.n > 0) {
    g.h_asum.resize((size_t)g.n);
    e = hipMemcpy(g.h_asum.data(), g.asum, sizeof(int64_t) * (size_t)g.n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      g.h_asum.clear();
      return hip_status(e, "copy neighbour-degree sums");
    }
  }
  if (g.h_qa.empty() && g.n > 0) {
    g.h_qa.resize((size_t)g.n);
    e = hipMemcpy(g.h_qa.data(), g.qa, sizeof(longlong2) * (size_t)g.n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      g.h_qa.clear();
      return hip_status(e, "copy neighbour-degree moments");
    }
  }
  // N_3(s) is the two-event degree sum D_2(s), at most its triangle-free
  // closed form; every cluster degree is below k_s + 3 k_max
  auto n3_bound = [&](int32_t v) {
    const double k = g.h_deg[v], A = (double)g.h_asum[v];
    const double Q = (double)g.h_qa[v].x, A2 = (double)g.h_qa[v].y;
    return std::max(0.0, k * (k - 4) * (k - 2) + (3 * k - 7) * A + Q + A2 - k * k);
  };
  const bool all = seeds == nullptr;
  std::vector<int32_t> useeds, inv;
  if (!all) {
    useeds.assign(seeds, seeds + n_seeds);
    std::sort(useeds.begin(), useeds.end());
    useeds.erase(std::unique(useeds.begin(), useeds.end()), useeds.end());
    inv.resize((size_t)n_seeds);
    for (int32_t i = 0; i < n_seeds; ++i)
      inv[i] = (int32_t)(std::lower_bound(useeds.begin(), useeds.end(), seeds[i]) - useeds.begin());
  }
  const int32_t n_work = all ? g.n : (int32_t)useeds.size();
  const double dmax = (double)g.info.max_degree;
  for (int32_t i = 0; i < n_work; ++i) {
    const int32_t v = all ? i : useeds[i];
    if (n3_bound(v) * ((double)g.h_deg[v] + 3 * dmax) > 4.0e18) {
      set_error("ef_compute_j3: the sums of seed %d (degree %d) could exceed int64", v,
                g.h_deg[v]);
      return EF_ERR_OVERFLOW;
    }
  }
  // items: the arcs of the seeds, largest seeds first
  auto order_of = [&](std::vector<int32_t> &ord, std::vector<int64_t> &off) {
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t c) {
      const double wa = n3_bound(a), wc = n3_bound(c);
      return wa != wc ? wa > wc : a < c;
    });
    off.assign(ord.size() + 1, 0);
    for (size_t i = 0; i < ord.size(); ++i) off[i + 1] = off[i] + g.h_deg[ord[i]];
  };
  const int64_t nnz = std::max<int64_t>(g.nnz, 1);
  if ((s = ws_ensure(g, WS_J3P, (2 * sizeof(long long) + sizeof(double)) * (size_t)nnz,
                     "per-arc partial sums")) != EF_OK)
    return s;
  long long *PN = (long long *)g.ws[WS_J3P].p, *PD = PN + nnz;
  double *PS = (double *)(PD + nnz);
  const int32_t *d_ord = nullptr;
  const int64_t *d_off = nullptr;
  int64_t n_items = 0;
  int32_t *d_useeds = nullptr;
  if (all) {
    if (!g.j3_seeds) {
      std::vector<int32_t> ord((size_t)g.n);
      std::iota(ord.begin(), ord.end(), 0);
      std::vector<int64_t> off;
      order_of(ord, off);
      if ((s = dev_alloc(g, (void **)&g.j3_seeds, sizeof(int32_t) * ord.size(), "j3 order")) !=
          EF_OK)
        return s;
      if ((s = dev_alloc(g, (void **)&g.j3_off, sizeof(int64_t) * off.size(), "j3 offsets")) !=
          EF_OK)
        return s;
      e = hipMemcpy(g.j3_seeds, ord.data(), sizeof(int32_t) * ord.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(g.j3_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_status(e, "upload j3 order");
    }
    d_ord = g.j3_seeds;
    d_off = g.j3_off;
    n_items = g.nnz;
  } else {
    std::vector<int32_t> ord(useeds);
    std::vector<int64_t> off;
    order_of(ord, off);
    n_items = off.back();
    const size_t bytes = sizeof(int64_t) * off.size() + sizeof(int32_t) * (2 * useeds.size()) + 64;
    if ((s = ws_ensure(g, WS_J3, bytes, "j3 seed lists")) != EF_OK) return s;
    int64_t *po = (int64_t *)g.ws[WS_J3].p;
    int32_t *pord = (int32_t *)(po + off.size());
    d_useeds = pord + ord.size();
    e = hipMemcpyAsync(po, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(pord, ord.data(), sizeof(int32_t) * ord.size(), hipMemcpyHostToDevice,
                         st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_useeds, useeds.data(), sizeof(int32_t) * useeds.size(),
                         hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_status(e, "upload seeds");
    d_ord = pord;
    d_off = po;
  }
  // outputs of the unique work list (staging unless they can go straight to
  // the caller's device arrays) and flag bytes
  const size_t out_bytes = (sizeof(double) + 2 * sizeof(int64_t)) * (size_t)std::max(n_work, 1);
  if ((s = ws_ensure(g, WS_UOUT, out_bytes, "output staging")) != EF_OK) return s;
  if ((s = ws_ensure(g, WS_FLAG, (sizeof(int32_t) + 1) * (size_t)std::max(n_work, 1),
                     "flag list")) != EF_OK)
    return s;
  double *ef_w = (double *)g.ws[WS_UOUT].p;
  int64_t *D_w = (int64_t *)(ef_w + std::max(n_work, 1)), *N_w = D_w + std::max(n_work, 1);
  if (all && out_dev) {
    ef_w = ef;
    if (D) D_w = D;
    if (N) N_w = N;
  }
  int32_t *fpos = (int32_t *)g.ws[WS_FLAG].p;
  uint8_t *fl = (uint8_t *)(fpos + std::max(n_work, 1));
  // per-bin item lists and their counts
  if ((s = ws_ensure(g, WS_J3L, sizeof(int32_t) * (5 * (size_t)std::max<int64_t>(n_items, 1) + 8),
                     "item lists")) != EF_OK)
    return s;
  int32_t *j3_lists = (int32_t *)g.ws[WS_J3L].p;
  int32_t *j3_counts = j3_lists + 5 * std::max<int64_t>(n_items, 1);
  const bool fp64 = prec == EF_PREC_FP64;
  prof.mark(0);
  e = launch_j3_items(g, fp64, d_ord, d_off, n_work, n_items, j3_lists, j3_counts, PN, PD, PS,
                      st);
  if (e != hipSuccess) return hip_status(e, "three-event items");
  prof.mark(1);
  e = launch_j3_finish(g, fp64, PN, PD, PS, d_useeds, nullptr, n_work, ef_w, D_w, N_w,
                       fp64 ? nullptr : fl, st);
  if (e != hipSuccess) return hip_status(e, "three-event finalize");
  prof.mark(2);
  int32_t n_flag = 0;
  if (!fp64) {
    // seeds whose FP32 EF cancels: their items again in FP64
    std::vector<uint8_t> hf((size_t)n_work);
    e = hipMemcpyAsync(hf.data(), fl, (size_t)n_work, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e, "read flags");
    std::vector<int32_t> fpos_h, ford;
    for (int32_t i = 0; i < n_work; ++i)
      if (hf[i]) {
        fpos_h.push_back(i);
        ford.push_back(all ? i : useeds[i]);
      }
    n_flag = (int32_t)fpos_h.size();
    if (n_flag > 0) {
      std::vector<int64_t> foff;
      order_of(ford, foff);
      const size_t bytes = sizeof(int64_t) * foff.size() + sizeof(int32_t) * ford.size() + 64;
      if ((s = ws_ensure(g, WS_SEEDS, bytes, "promoted seeds")) != EF_OK) return s;
      int64_t *po = (int64_t *)g.ws[WS_SEEDS].p;
      int32_t *pord = (int32_t *)(po + foff.size());
      e = hipMemcpyAsync(po, foff.data(), sizeof(int64_t) * foff.size(), hipMemcpyHostToDevice,
                         st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(pord, ford.data(), sizeof(int32_t) * ford.size(),
                           hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(fpos, fpos_h.data(), sizeof(int32_t) * fpos_h.size(),
                           hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = launch_j3_items(g, true, pord, po, n_flag, foff.back(), j3_lists, j3_counts, PN, PD,
                            PS, st);
      if (e == hipSuccess)
        e = launch_j3_finish(g, true, PN, PD, PS, d_useeds, fpos, n_flag, ef_w, D_w, N_w,
                             nullptr, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_status(e, "three-event FP64 recompute");
    }
  }
  prof.mark(3);
  // deliver outputs
  if (!all) {
    if (out_dev) {
      if ((s = ws_ensure(g, WS_SEEDS, sizeof(int32_t) * inv.size() + 64, "inverse map")) != EF_OK)
        return s;
      int32_t *d_inv = (int32_t *)g.ws[WS_SEEDS].p;
      e = hipMemcpyAsync(d_inv, inv.data(), sizeof(int32_t) * inv.size(), hipMemcpyHostToDevice,
                         st);
      if (e == hipSuccess) e = launch_gather_outputs(d_inv, n_seeds, ef_w, D_w, N_w, ef, D, N, st);
      if (e != hipSuccess) return hip_status(e, "scatter outputs");
    } else {
      std::vector<double> hef((size_t)n_work);
      std::vector<int64_t> hD((size_t)n_work), hN((size_t)n_work);
      e = hipMemcpyAsync(hef.data(), ef_w, sizeof(double) * n_work, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hD.data(), D_w, sizeof(int64_t) * n_work, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hN.data(), N_w, sizeof(int64_t) * n_work, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_status(e, "copy outputs");
      for (int32_t i = 0; i < n_seeds; ++i) {
        ef[i] = hef[inv[i]];
        if (D) D[i] = hD[inv[i]];
        if (N) N[i] = hN[inv[i]];
      }
    }
  } else if (!out_dev) {
    e = hipMemcpyAsync(ef, ef_w, sizeof(double) * (size_t)g.n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && D)
      e = hipMemcpyAsync(D, D_w, sizeof(int64_t) * (size_t)g.n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && N)
      e = hipMemcpyAsync(N, N_w, sizeof(int64_t) * (size_t)g.n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e, "copy outputs");
  }
  g.stats.seeds = n_work;
  g.stats.promoted = n_flag;
  if (prof.on) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e, "profile");
    g.stats.t_stream_ms = prof.ms(0, 1);
    g.stats.t_finalize_ms = prof.ms(1, 2);
    g.stats.t_pass2_ms = prof.ms(2, 3);
    g.stats.t_total_ms = prof.ms(0, 3);
  }
  return EF_OK;
}

// Top-k over device EF values of the graph's nodes, in the handle's workspace;
// host outputs go through a device staging area after the top-k scratch.
static ef_status topk_device_values(Graph &g, const double *ef_all, int32_t k, int32_t *nodes,
                                    double *ef, bool out_dev, hipStream_t st) {
  const size_t sort_bytes = (topk_scratch_bytes(g.n, k) + 255) & ~(size_t)255;
  const size_t node_bytes = (sizeof(int32_t) * (size_t)k + 255) & ~(size_t)255;
  const size_t stage = out_dev ? 0 : node_bytes + sizeof(double) * (size_t)k;
  ef_status s = ws_ensure(g, WS_TOPK, sort_bytes + stage, "top-k scratch");
  if (s != EF_OK) return s;
  char *base = (char *)g.ws[WS_TOPK].p;
  int32_t *nodes_d = nodes;
  double *ef_d = ef;
  if (!out_dev) {
    nodes_d = (int32_t *)(base + sort_bytes);
    ef_d = (double *)(base + sort_bytes + node_bytes);
  }
  hipError_t e = launch_topk(ef_all, g.n, k, base, sort_bytes, nodes_d, ef ? ef_d : nullptr, st);
  if (e != hipSuccess) return hip_status(e, "top-k");
  if (!out_dev) {
    e = hipMemcpyAsync(nodes, nodes_d, sizeof(int32_t) * (size_t)k, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && ef)
      e = hipMemcpyAsync(ef, ef_d, sizeof(double) * (size_t)k, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e, "copy top-k");
  }
  return EF_OK;
}

extern "C" ef_status ef_topk(ef_graph *h, ef_algo algo, ef_prec prec, int32_t k, int32_t *nodes,
                             double *ef, uint32_t flags, void *hip_stream) {
  if (!h || !nodes) {
    set_error("ef_topk: null handle or output");
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  if (k < 0 || k > g.n) {
    set_error("ef_topk: k=%d outside [0, n=%d]", k, g.n);
    return EF_ERR_ARG;
  }
  if (flags & ~(EF_OUT_DEVICE | EF_PROFILE)) {
    set_error("ef_topk: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  if (k == 0) return EF_OK;
  const size_t n = (size_t)g.n;
  ef_status s = ws_ensure(g, WS_OUT, sizeof(double) * n + 2 * sizeof(int64_t) * n + 2048,
                          "all-node outputs");
  if (s != EF_OK) return s;
  double *ef_all = (double *)g.ws[WS_OUT].p;
  int64_t *D_all = (int64_t *)(ef_all + n);
  int64_t *N_all = D_all + n;
  s = ef_compute(h, algo, prec, nullptr, 0, ef_all, D_all, N_all,
                 EF_OUT_DEVICE | (flags & EF_PROFILE), hip_stream);
  if (s != EF_OK) return s;
  return topk_device_values(g, ef_all, k, nodes, ef, (flags & EF_OUT_DEVICE) != 0,
                            (hipStream_t)hip_stream);
}

extern "C" ef_status ef_topk_values(ef_graph *h, const double *ef_in, int32_t k, int32_t *nodes,
                                    double *ef, uint32_t flags, void *hip_stream) {
  if (!h || !nodes || (!ef_in && k > 0)) {
    set_error("ef_topk_values: null handle, values or output");
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  if (k < 0 || k > g.n) {
    set_error("ef_topk_values: k=%d outside [0, n=%d]", k, g.n);
    return EF_ERR_ARG;
  }
  if (flags & ~EF_OUT_DEVICE) {
    set_error("ef_topk_values: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  if (k == 0) return EF_OK;
  return topk_device_values(g, ef_in, k, nodes, ef, (flags & EF_OUT_DEVICE) != 0,
                            (hipStream_t)hip_stream);
}
