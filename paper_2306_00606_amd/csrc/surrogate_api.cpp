// C-ABI of the learned surrogate: parameters, features, GPU training,
// prediction, and the surrogate-accelerated top-k with the exact kernel as
// rescoring step, judge and fallback.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <random>
#include <vector>

#include "ef_internal.h"

namespace efi {
hipError_t launch_features(const Graph &g, const float *mean, const float *inv_std, float *X,
                           float *lnN, hipStream_t st);
hipError_t launch_mlp_pack(const float *P, __bf16 *pack, hipStream_t st);
hipError_t launch_mlp_forward(const float *X, int64_t rows, const float *P, const __bf16 *pack,
                              const float *lnN, float *y, double *ef, hipStream_t st);
hipError_t launch_mlp_grad(const float *X, const float *Yt, const int32_t *perm, int64_t b0,
                           int64_t nrows, const float *P, const __bf16 *pack, float *part,
                           float *part_loss, int32_t nblocks, float *grad, float *loss,
                           hipStream_t st);
hipError_t launch_adam(float *P, float *M, float *V, const float *grad, float lr, float b1,
                       float b2, float eps, float wd, int32_t t, hipStream_t st);
int32_t mlp_param_count();
int32_t mlp_pack_count();
}  // namespace efi

using namespace efi;

extern "C" ef_status ef_compute(ef_graph *g, ef_algo algo, ef_prec prec, const int32_t *seeds,
                                int32_t n_seeds, double *ef, int64_t *D, int64_t *N,
                                uint32_t flags, void *hip_stream);
extern "C" ef_status ef_topk(ef_graph *g, ef_algo algo, ef_prec prec, int32_t k, int32_t *nodes,
                             double *ef, uint32_t flags, void *hip_stream);

constexpr int kNF = 16;
constexpr int kMaxGradBlocks = 64;

struct ef_surrogate {
  std::vector<float> P, M, V;  // FP32 masters and Adam moments (host copies)
  float mean[kNF] = {}, inv_std[kNF] = {};
  int32_t step = 0;
  // device mirrors
  float *dP = nullptr, *dM = nullptr, *dV = nullptr, *dgrad = nullptr, *dloss = nullptr;
  float *dpart = nullptr, *dpart_loss = nullptr, *dmean = nullptr, *dinv = nullptr;
  __bf16 *dpack = nullptr;
  bool device_ready = false;
  bool host_dirty = false;  // device holds newer parameters than the host copy
};

static ef_status sg_device(ef_surrogate *s) {
  if (s->device_ready) return EF_OK;
  const size_t np = (size_t)mlp_param_count();
  hipError_t e = hipMalloc(&s->dP, sizeof(float) * np);
  if (e == hipSuccess) e = hipMalloc(&s->dM, sizeof(float) * np);
  if (e == hipSuccess) e = hipMalloc(&s->dV, sizeof(float) * np);
  if (e == hipSuccess) e = hipMalloc(&s->dgrad, sizeof(float) * np);
  if (e == hipSuccess) e = hipMalloc(&s->dloss, sizeof(float) * 4);
  if (e == hipSuccess) e = hipMalloc(&s->dpart, sizeof(float) * np * kMaxGradBlocks * 4);
  if (e == hipSuccess) e = hipMalloc(&s->dpart_loss, sizeof(float) * kMaxGradBlocks * 4);
  if (e == hipSuccess) e = hipMalloc(&s->dmean, sizeof(float) * kNF);
  if (e == hipSuccess) e = hipMalloc(&s->dinv, sizeof(float) * kNF);
  if (e == hipSuccess) e = hipMalloc(&s->dpack, sizeof(__bf16) * (size_t)mlp_pack_count());
  if (e != hipSuccess) return hip_status(e, "surrogate device buffers");
  s->device_ready = true;
  return EF_OK;
}

// host -> device (parameters, moments, standardisation) and re-pack
static ef_status sg_upload(ef_surrogate *s, hipStream_t st) {
  ef_status r = sg_device(s);
  if (r != EF_OK) return r;
  const size_t np = (size_t)mlp_param_count();
  hipError_t e = hipMemcpyAsync(s->dP, s->P.data(), sizeof(float) * np, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s->dM, s->M.data(), sizeof(float) * np, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s->dV, s->V.data(), sizeof(float) * np, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s->dmean, s->mean, sizeof(float) * kNF, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s->dinv, s->inv_std, sizeof(float) * kNF, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_mlp_pack(s->dP, s->dpack, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return hip_status(e, "upload surrogate");
}

static ef_status sg_download(ef_surrogate *s, hipStream_t st) {
  if (!s->host_dirty) return EF_OK;
  const size_t np = (size_t)mlp_param_count();
  hipError_t e = hipMemcpyAsync(s->P.data(), s->dP, sizeof(float) * np, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s->M.data(), s->dM, sizeof(float) * np, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s->V.data(), s->dV, sizeof(float) * np, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_status(e, "download surrogate");
  s->host_dirty = false;
  return EF_OK;
}

extern "C" {

ef_status ef_surrogate_create(uint64_t seed, ef_surrogate **out) {
  if (!out) {
    set_error("ef_surrogate_create: null output");
    return EF_ERR_ARG;
  }
  ef_surrogate *s = new (std::nothrow) ef_surrogate();
  if (!s) {
    set_error("host allocation failed");
    return EF_ERR_NOMEM;
  }
  const int np = mlp_param_count();
  s->P.assign(np, 0.f);
  s->M.assign(np, 0.f);
  s->V.assign(np, 0.f);
  // He-style normal initialisation of the weights, zero biases
  std::mt19937_64 rng(seed);
  std::normal_distribution<float> nd(0.f, 1.f);
  for (int i = 0; i < 1024; ++i) s->P[i] = nd(rng) * std::sqrt(2.0f / 16.0f);
  for (int i = 1088; i < 5184; ++i) s->P[i] = nd(rng) * std::sqrt(2.0f / 64.0f);
  for (int i = 5248; i < 5312; ++i) s->P[i] = nd(rng) * std::sqrt(1.0f / 64.0f);
  for (int i = 0; i < kNF; ++i) {
    s->mean[i] = 0.f;
    s->inv_std[i] = 1.f;
  }
  *out = s;
  return EF_OK;
}

ef_status ef_surrogate_free(ef_surrogate *s) {
  if (!s) {
    set_error("ef_surrogate_free: null handle");
    return EF_ERR_ARG;
  }
  for (void *p : {(void *)s->dP, (void *)s->dM, (void *)s->dV, (void *)s->dgrad, (void *)s->dloss,
                  (void *)s->dpart, (void *)s->dpart_loss, (void *)s->dmean, (void *)s->dinv,
                  (void *)s->dpack})
    if (p) (void)hipFree(p);
  delete s;
  return EF_OK;
}

ef_status ef_surrogate_get_params(ef_surrogate *s, float *params, float *mean, float *inv_std) {
  if (!s) {
    set_error("ef_surrogate_get_params: null handle");
    return EF_ERR_ARG;
  }
  ef_status r = sg_download(s, nullptr);
  if (r != EF_OK) return r;
  if (params) std::memcpy(params, s->P.data(), sizeof(float) * s->P.size());
  if (mean) std::memcpy(mean, s->mean, sizeof(s->mean));
  if (inv_std) std::memcpy(inv_std, s->inv_std, sizeof(s->inv_std));
  return EF_OK;
}

ef_status ef_surrogate_set_params(ef_surrogate *s, const float *params, const float *mean,
                                  const float *inv_std) {
  if (!s) {
    set_error("ef_surrogate_set_params: null handle");
    return EF_ERR_ARG;
  }
  if (params) std::memcpy(s->P.data(), params, sizeof(float) * s->P.size());
  if (mean) std::memcpy(s->mean, mean, sizeof(s->mean));
  if (inv_std) std::memcpy(s->inv_std, inv_std, sizeof(s->inv_std));
  std::fill(s->M.begin(), s->M.end(), 0.f);
  std::fill(s->V.begin(), s->V.end(), 0.f);
  s->step = 0;
  s->host_dirty = false;
  if (s->device_ready) return sg_upload(s, nullptr);
  return EF_OK;
}

static const char kMagic[8] = {'E', 'F', 'S', 'G', '0', '0', '0', '1'};

ef_status ef_surrogate_save(ef_surrogate *s, const char *path) {
  if (!s || !path) {
    set_error("ef_surrogate_save: null argument");
    return EF_ERR_ARG;
  }
  ef_status r = sg_download(s, nullptr);
  if (r != EF_OK) return r;
  FILE *f = std::fopen(path, "wb");
  if (!f) {
    set_error("cannot open %s for writing", path);
    return EF_ERR_ARG;
  }
  const int32_t np = mlp_param_count();
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 &&
            std::fwrite(&s->step, 4, 1, f) == 1 &&
            std::fwrite(s->P.data(), 4, np, f) == (size_t)np &&
            std::fwrite(s->M.data(), 4, np, f) == (size_t)np &&
            std::fwrite(s->V.data(), 4, np, f) == (size_t)np &&
            std::fwrite(s->mean, 4, kNF, f) == (size_t)kNF &&
            std::fwrite(s->inv_std, 4, kNF, f) == (size_t)kNF;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) {
    set_error("write to %s failed", path);
    return EF_ERR_ARG;
  }
  return EF_OK;
}

ef_status ef_surrogate_load(ef_surrogate *s, const char *path) {
  if (!s || !path) {
    set_error("ef_surrogate_load: null argument");
    return EF_ERR_ARG;
  }
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    set_error("cannot open %s", path);
    return EF_ERR_ARG;
  }
  char magic[8];
  int32_t np = 0, step = 0;
  const int32_t want = mlp_param_count();
  std::vector<float> P(want), M(want), V(want);
  float mean[kNF], inv[kNF];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
            std::fread(&np, 4, 1, f) == 1 && np == want && std::fread(&step, 4, 1, f) == 1 &&
            std::fread(P.data(), 4, np, f) == (size_t)np &&
            std::fread(M.data(), 4, np, f) == (size_t)np &&
            std::fread(V.data(), 4, np, f) == (size_t)np &&
            std::fread(mean, 4, kNF, f) == (size_t)kNF && std::fread(inv, 4, kNF, f) == (size_t)kNF;
  std::fclose(f);
  if (!ok) {
    set_error("%s is not a surrogate file of this version", path);
    return EF_ERR_ARG;
  }
  s->P = P;
  s->M = M;
  s->V = V;
  std::memcpy(s->mean, mean, sizeof(mean));
  std::memcpy(s->inv_std, inv, sizeof(inv));
  s->step = step;
  s->host_dirty = false;
  if (s->device_ready) return sg_upload(s, nullptr);
  return EF_OK;
}

ef_status ef_features(ef_graph *h, float *X, float *lnN, uint32_t flags, void *hip_stream) {
  if (!h || !X) {
    set_error("ef_features: null argument");
    return EF_ERR_ARG;
  }
  if (flags & ~EF_OUT_DEVICE) {
    set_error("ef_features: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  if (g.n == 0) return EF_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t n = (size_t)g.n;
  char *p = nullptr;
  const size_t need = (sizeof(float) * kNF + sizeof(float)) * n + 4096;
  ef_status rs = graph_scratch(g, need, (void **)&p);
  if (rs != EF_OK) return rs;
  hipError_t e = hipSuccess;
  auto take = [&](size_t b) {
    char *r = p;
    p += (b + 255) & ~(size_t)255;
    return r;
  };
  char *base = p;
  const bool dev = (flags & EF_OUT_DEVICE) != 0;
  float *Xd = dev ? X : (float *)take(sizeof(float) * kNF * n);
  float *Ld = (dev && lnN) ? lnN : (float *)take(sizeof(float) * n);
  e = launch_features(g, nullptr, nullptr, Xd, Ld, st);
  if (e == hipSuccess && !dev) {
    e = hipMemcpyAsync(X, Xd, sizeof(float) * kNF * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && lnN) e = hipMemcpyAsync(lnN, Ld, sizeof(float) * n, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)base;
  return hip_status(e, "features");
}

ef_status ef_surrogate_gradients(ef_surrogate *s, const float *X, const float *y, int64_t rows,
                                 float *grad, float *loss, void *hip_stream) {
  if (!s || !X || !y || rows <= 0 || !grad) {
    set_error("ef_surrogate_gradients: bad arguments");
    return EF_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  ef_status r = sg_download(s, st);
  if (r == EF_OK) r = sg_upload(s, st);
  if (r != EF_OK) return r;
  float *dX = nullptr, *dy = nullptr;
  int32_t *dperm = nullptr;
  hipError_t e = hipMalloc(&dX, sizeof(float) * kNF * rows);
  if (e == hipSuccess) e = hipMalloc(&dy, sizeof(float) * rows);
  if (e == hipSuccess) e = hipMalloc(&dperm, sizeof(int32_t) * rows);
  std::vector<int32_t> perm((size_t)rows);
  std::iota(perm.begin(), perm.end(), 0);
  if (e == hipSuccess) e = hipMemcpyAsync(dX, X, sizeof(float) * kNF * rows, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dy, y, sizeof(float) * rows, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dperm, perm.data(), sizeof(int32_t) * rows, hipMemcpyHostToDevice, st);
  const int64_t tiles = (rows + 31) / 32;
  const int32_t nblocks = (int32_t)std::min<int64_t>((tiles + 3) / 4, kMaxGradBlocks);
  if (e == hipSuccess)
    e = launch_mlp_grad(dX, dy, dperm, 0, rows, s->dP, s->dpack, s->dpart, s->dpart_loss, nblocks,
                        s->dgrad, s->dloss, st);
  float hl = 0.f;
  if (e == hipSuccess)
    e = hipMemcpyAsync(grad, s->dgrad, sizeof(float) * mlp_param_count(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&hl, s->dloss, sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dX);
  (void)hipFree(dy);
  (void)hipFree(dperm);
  if (loss) *loss = hl / (float)rows;
  return hip_status(e, "surrogate gradients");
}

ef_status ef_surrogate_forward(ef_surrogate *s, const float *X, int64_t rows, float *y,
                               uint32_t flags, void *hip_stream) {
  if (!s || rows < 0 || (rows > 0 && (!X || !y))) {
    set_error("ef_surrogate_forward: bad arguments");
    return EF_ERR_ARG;
  }
  if (flags & ~EF_OUT_DEVICE) {
    set_error("ef_surrogate_forward: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  if (rows == 0) return EF_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  ef_status r = s->device_ready ? EF_OK : sg_upload(s, st);
  if (r != EF_OK) return r;
  if (flags & EF_OUT_DEVICE)
    return hip_status(launch_mlp_forward(X, rows, s->dP, s->dpack, nullptr, y, nullptr, st),
                      "surrogate forward");
  float *dX = nullptr, *dy = nullptr;
  hipError_t e = hipMalloc(&dX, sizeof(float) * kNF * rows);
  if (e == hipSuccess) e = hipMalloc(&dy, sizeof(float) * rows);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dX, X, sizeof(float) * kNF * rows, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_mlp_forward(dX, rows, s->dP, s->dpack, nullptr, dy, nullptr, st);
  if (e == hipSuccess) e = hipMemcpyAsync(y, dy, sizeof(float) * rows, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dX);
  (void)hipFree(dy);
  return hip_status(e, "surrogate forward");
}

ef_status ef_surrogate_train(ef_surrogate *s, const float *X, const float *y, int64_t rows,
                             const ef_train_cfg *cfg, ef_train_report *rep, void *hip_stream) {
  if (!s || !X || !y || rows < 64 || !cfg || cfg->epochs < 0 || cfg->batch < 32 ||
      !(cfg->lr > 0.f) || cfg->val_fraction < 0.f || cfg->val_fraction >= 0.9f ||
      !(cfg->lr_end > 0.f && cfg->lr_end <= 1.f)) {
    set_error("ef_surrogate_train: bad arguments");
    return EF_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  ef_status r = sg_download(s, st);
  if (r != EF_OK) return r;
  // standardisation from the data (FP64 sums on the host)
  for (int f = 0; f < kNF; ++f) {
    double m = 0.0, q = 0.0;
    for (int64_t i = 0; i < rows; ++i) m += X[i * kNF + f];
    m /= (double)rows;
    for (int64_t i = 0; i < rows; ++i) {
      const double d = X[i * kNF + f] - m;
      q += d * d;
    }
    const double sd = std::sqrt(q / (double)rows);
    s->mean[f] = (float)m;
    s->inv_std[f] = (float)(sd > 1e-6 ? 1.0 / sd : 1.0);
  }
  std::vector<float> Xs((size_t)rows * kNF);
  for (int64_t i = 0; i < rows; ++i)
    for (int f = 0; f < kNF; ++f)
      Xs[i * kNF + f] = (X[i * kNF + f] - s->mean[f]) * s->inv_std[f];
  // split
  std::mt19937_64 rng(cfg->seed);
  std::vector<int32_t> idx((size_t)rows);
  std::iota(idx.begin(), idx.end(), 0);
  std::shuffle(idx.begin(), idx.end(), rng);
  const int64_t nval = (int64_t)(cfg->val_fraction * (double)rows);
  const int64_t ntr = rows - nval;
  if ((r = sg_upload(s, st)) != EF_OK) return r;
  float *dX = nullptr, *dy = nullptr, *dbest = nullptr;
  int32_t *dperm = nullptr, *dval = nullptr;
  const size_t np = (size_t)mlp_param_count();
  hipError_t e = hipMalloc(&dX, sizeof(float) * kNF * rows);
  if (e == hipSuccess) e = hipMalloc(&dy, sizeof(float) * rows);
  if (e == hipSuccess) e = hipMalloc(&dperm, sizeof(int32_t) * std::max<int64_t>(ntr, 1));
  if (e == hipSuccess) e = hipMalloc(&dval, sizeof(int32_t) * std::max<int64_t>(nval, 1));
  if (e == hipSuccess) e = hipMalloc(&dbest, sizeof(float) * np);
  if (e == hipSuccess) e = hipMemcpyAsync(dX, Xs.data(), sizeof(float) * kNF * rows, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dy, y, sizeof(float) * rows, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && nval > 0)
    e = hipMemcpyAsync(dval, idx.data() + ntr, sizeof(int32_t) * nval, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dbest, s->dP, sizeof(float) * np, hipMemcpyDeviceToDevice, st);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e == hipSuccess) e = hipEventRecord(t0, st);
  std::vector<int32_t> tr(idx.begin(), idx.begin() + ntr);
  float best = INFINITY, last_train = 0.f, last_val = 0.f;
  int32_t since_best = 0, epochs_run = 0;
  const int64_t batch = cfg->batch;
  // step size: a half cosine from lr (first step) to lr * lr_end (last step
  // of the configured epochs)
  const int64_t steps_total = (int64_t)cfg->epochs * ((ntr + batch - 1) / batch);
  int64_t t_step = 0;
  const auto step_lr = [&](int64_t t) {
    const double u = steps_total > 1 ? (double)t / (double)(steps_total - 1) : 1.0;
    const double f = cfg->lr_end + (1.0 - cfg->lr_end) * 0.5 * (1.0 + std::cos(M_PI * u));
    return (float)(cfg->lr * f);
  };
  for (int32_t ep = 0; ep < cfg->epochs && e == hipSuccess; ++ep) {
    std::shuffle(tr.begin(), tr.end(), rng);
    e = hipMemcpyAsync(dperm, tr.data(), sizeof(int32_t) * ntr, hipMemcpyHostToDevice, st);
    double tl = 0.0;
    for (int64_t b0 = 0; b0 < ntr && e == hipSuccess; b0 += batch) {
      const int64_t nb = std::min(batch, ntr - b0);
      const int64_t tiles = (nb + 31) / 32;
      const int32_t nblocks = (int32_t)std::min<int64_t>((tiles + 3) / 4, kMaxGradBlocks);
      e = launch_mlp_grad(dX, dy, dperm, b0, nb, s->dP, s->dpack, s->dpart, s->dpart_loss,
                          nblocks, s->dgrad, s->dloss, st);
      if (e == hipSuccess)
        e = launch_adam(s->dP, s->dM, s->dV, s->dgrad, step_lr(t_step++), 0.9f, 0.999f, 1e-8f,
                        cfg->weight_decay, ++s->step, st);
      if (e == hipSuccess) e = launch_mlp_pack(s->dP, s->dpack, st);
    }
    // training loss of the epoch's last state and validation loss
    float hl = 0.f;
    if (e == hipSuccess && nval > 0) {
      const int64_t tiles = (nval + 31) / 32;
      const int32_t nblocks = (int32_t)std::min<int64_t>((tiles + 3) / 4, kMaxGradBlocks);
      e = launch_mlp_grad(dX, dy, dval, 0, nval, s->dP, s->dpack, s->dpart, s->dpart_loss,
                          nblocks, s->dgrad, s->dloss, st);
      if (e == hipSuccess) e = hipMemcpyAsync(&hl, s->dloss, sizeof(float), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      last_val = hl / (float)nval;
    }
    (void)tl;
    ++epochs_run;
    const float score = nval > 0 ? last_val : (float)ep;
    if (nval > 0 && score < best) {
      best = score;
      since_best = 0;
      if (e == hipSuccess)
        e = hipMemcpyAsync(dbest, s->dP, sizeof(float) * np, hipMemcpyDeviceToDevice, st);
    } else if (nval > 0 && ++since_best > cfg->patience) {
      break;
    }
  }
  // training loss over all training rows at the end
  if (e == hipSuccess && nval > 0) {
    e = hipMemcpyAsync(s->dP, dbest, sizeof(float) * np, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = launch_mlp_pack(s->dP, s->dpack, st);
  }
  if (e == hipSuccess) {
    const int64_t tiles = (ntr + 31) / 32;
    const int32_t nblocks = (int32_t)std::min<int64_t>((tiles + 3) / 4, kMaxGradBlocks);
    std::vector<int32_t> ordered(tr);
    e = hipMemcpyAsync(dperm, ordered.data(), sizeof(int32_t) * ntr, hipMemcpyHostToDevice, st);
    float hl = 0.f;
    if (e == hipSuccess)
      e = launch_mlp_grad(dX, dy, dperm, 0, ntr, s->dP, s->dpack, s->dpart, s->dpart_loss,
                          nblocks, s->dgrad, s->dloss, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hl, s->dloss, sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(t1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    last_train = hl / (float)ntr;
  }
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(dX);
  (void)hipFree(dy);
  (void)hipFree(dperm);
  (void)hipFree(dval);
  (void)hipFree(dbest);
  if (e != hipSuccess) return hip_status(e, "surrogate training");
  s->host_dirty = true;
  if (rep) {
    rep->epochs_run = epochs_run;
    rep->train_loss = last_train;
    rep->val_loss = nval > 0 ? best : 0.f;
    rep->train_ms = ms;
    rep->rows = rows;
    rep->val_rows = nval;
  }
  return EF_OK;
}

ef_status ef_surrogate_predict(ef_surrogate *s, ef_graph *h, double *ef_pred, uint32_t flags,
                               void *hip_stream) {
  if (!s || !h || !ef_pred) {
    set_error("ef_surrogate_predict: null argument");
    return EF_ERR_ARG;
  }
  if (flags & ~EF_OUT_DEVICE) {
    set_error("ef_surrogate_predict: unknown flags 0x%x", flags);
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  if (g.n == 0) return EF_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  ef_status r = s->device_ready ? EF_OK : sg_upload(s, st);
  if (r != EF_OK) return r;
  const size_t n = (size_t)g.n;
  char *p = nullptr;
  const size_t need = (sizeof(float) * kNF + sizeof(float)) * n + sizeof(double) * n + 4096;
  ef_status rs = graph_scratch(g, need, (void **)&p);
  if (rs != EF_OK) return rs;
  hipError_t e = hipSuccess;
  char *base = p;
  auto take = [&](size_t b) {
    char *rr = p;
    p += (b + 255) & ~(size_t)255;
    return rr;
  };
  float *Xd = (float *)take(sizeof(float) * kNF * n);
  float *Ld = (float *)take(sizeof(float) * n);
  const bool dev = (flags & EF_OUT_DEVICE) != 0;
  double *Ed = dev ? ef_pred : (double *)take(sizeof(double) * n);
  e = launch_features(g, s->dmean, s->dinv, Xd, Ld, st);
  if (e == hipSuccess) e = launch_mlp_forward(Xd, (int64_t)n, s->dP, s->dpack, Ld, nullptr, Ed, st);
  if (e == hipSuccess && !dev)
    e = hipMemcpyAsync(ef_pred, Ed, sizeof(double) * n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && !dev) e = hipStreamSynchronize(st);
  (void)base;
  return hip_status(e, "surrogate predict");
}

}  // extern "C"

// Spearman correlation with average ranks for ties
static double spearman(const std::vector<double> &a, const std::vector<double> &b) {
  auto ranks = [](const std::vector<double> &v) {
    std::vector<int64_t> o(v.size());
    std::iota(o.begin(), o.end(), 0);
    std::stable_sort(o.begin(), o.end(), [&](int64_t x, int64_t y) { return v[x] < v[y]; });
    std::vector<double> r(v.size());
    size_t i = 0;
    while (i < o.size()) {
      size_t j = i;
      while (j + 1 < o.size() && v[o[j + 1]] == v[o[i]]) ++j;
      for (size_t t = i; t <= j; ++t) r[o[t]] = 0.5 * (double)(i + j);
      i = j + 1;
    }
    return r;
  };
  std::vector<double> ra = ranks(a), rb = ranks(b);
  const double n = (double)a.size();
  double ma = 0, mb = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    ma += ra[i];
    mb += rb[i];
  }
  ma /= n;
  mb /= n;
  double sab = 0, saa = 0, sbb = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    sab += (ra[i] - ma) * (rb[i] - mb);
    saa += (ra[i] - ma) * (ra[i] - ma);
    sbb += (rb[i] - mb) * (rb[i] - mb);
  }
  return (saa > 0 && sbb > 0) ? sab / std::sqrt(saa * sbb) : 0.0;
}

extern "C" ef_status ef_topk_surrogate(ef_graph *h, ef_surrogate *s, int32_t k,
                                       int32_t rerank_factor, int32_t judge_sample,
                                       float min_spearman, uint64_t seed, int32_t *nodes,
                                       double *ef_exact, ef_judge_report *rep,
                                       void *hip_stream) {
  if (!h || !s || !nodes || k < 0 || rerank_factor < 1 || judge_sample < 0) {
    set_error("ef_topk_surrogate: bad arguments");
    return EF_ERR_ARG;
  }
  Graph &g = h->g;
  if (k > g.n) {
    set_error("ef_topk_surrogate: k=%d > n=%d", k, g.n);
    return EF_ERR_ARG;
  }
  if (k == 0) return EF_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  hipEvent_t ev[4] = {};
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) return hip_status(hipErrorUnknown, "events");
  ef_judge_report R{};
  (void)hipEventRecord(ev[0], st);
  // 1) surrogate scores for every node
  std::vector<double> pred((size_t)g.n);
  ef_status r = ef_surrogate_predict(s, h, pred.data(), 0, hip_stream);
  (void)hipEventRecord(ev[1], st);
  // 2) exact rescoring of the best rerank_factor * k candidates
  const int32_t c = (int32_t)std::min<int64_t>((int64_t)k * rerank_factor, g.n);
  std::vector<int32_t> cand((size_t)g.n);
  std::iota(cand.begin(), cand.end(), 0);
  if (r == EF_OK) {
    std::partial_sort(cand.begin(), cand.begin() + c, cand.end(), [&](int32_t a, int32_t b) {
      return pred[a] != pred[b] ? pred[a] > pred[b] : a < b;
    });
    cand.resize((size_t)c);
  }
  std::vector<double> ex((size_t)c);
  if (r == EF_OK)
    r = ef_compute(h, EF_ALGO_PER_SEED, EF_PREC_FP32C, cand.data(), c, ex.data(), nullptr, nullptr,
                   0, hip_stream);
  (void)hipEventRecord(ev[2], st);
  // 3) judge: rank agreement of surrogate and exact EF on a random sample
  if (r == EF_OK && judge_sample > 0) {
    std::mt19937_64 rng(seed);
    const int32_t m = std::min(judge_sample, g.n);
    std::vector<int32_t> sample((size_t)m);
    for (auto &x : sample) x = (int32_t)(rng() % (uint64_t)g.n);
    std::vector<double> exs((size_t)m), ps((size_t)m);
    r = ef_compute(h, EF_ALGO_PER_SEED, EF_PREC_FP32C, sample.data(), m, exs.data(), nullptr,
                   nullptr, 0, hip_stream);
    for (int32_t i = 0; i < m; ++i) ps[i] = pred[sample[i]];
    R.sample = m;
    R.spearman = (float)spearman(ps, exs);
  }
  (void)hipEventRecord(ev[3], st);
  if (r == EF_OK && judge_sample > 0 && R.spearman < min_spearman) {
    // fallback: the exact top-k of the whole graph
    R.fallback = 1;
    r = ef_topk(h, EF_ALGO_CLUSTER, EF_PREC_FP32C, k, nodes, ef_exact, 0, hip_stream);
  } else if (r == EF_OK) {
    std::vector<int32_t> o((size_t)c);
    std::iota(o.begin(), o.end(), 0);
    std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) {
      return ex[a] != ex[b] ? ex[a] > ex[b] : cand[a] < cand[b];
    });
    for (int32_t i = 0; i < k; ++i) {
      nodes[i] = cand[o[i]];
      if (ef_exact) ef_exact[i] = ex[o[i]];
    }
  }
  if (hipStreamSynchronize(st) == hipSuccess) {
    float a = 0, b = 0, d = 0;
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[1], ev[2]);
    (void)hipEventElapsedTime(&d, ev[2], ev[3]);
    R.t_predict_ms = a;
    R.t_rescore_ms = b;
    R.t_judge_ms = d;
  }
  R.candidates = c;
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (rep) *rep = R;
  return r;
}
