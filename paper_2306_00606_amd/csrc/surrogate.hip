// Learned surrogate for Expected Force: per-node features, and a small MLP
// (16 -> 64 -> GELU -> 64 -> GELU -> 1, GELU in its tanh form) with BF16 operands and FP32
// accumulation on the gfx950 matrix cores (v_mfma_f32_32x32x16_bf16), trained
// on the GPU by its own forward and backward kernels and an Adam step.
//
// The network predicts the residual y = ln N(s) - EF(s) >= 0 (EF is at most
// ln N, with equality when all clusters of s have the same degree); the
// predicted EF is max(0, ln N - y).
//
// MFMA operand layouts (wave64, 32x32x16): lane l holds
//   A[i][k]  for i = l % 32, k = 8 (l / 32) + j          (8 bf16, j = 0..7)
//   B[k][n]  for n = l % 32, k = 8 (l / 32) + j          (8 bf16)
//   C[i][n]  for n = l % 32, i = 8 (r / 4) + 4 (l / 32) + r % 4  (16 fp32, r = 0..15)
// Weights are kept as FP32 masters and re-packed into the B layout (bf16)
// after every optimiser step.
#include "device_common.h"

namespace efi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kF = 16, kH = 64;
// flat parameter vector
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248,
              kOffB3 = 5312, kParams = 5313;
// packed bf16 B-operand blocks (64 lanes x 8 values each)
constexpr int kPackW1 = 0;                  // kb 1 x nb 2
constexpr int kPackW2 = 2;                  // kb 4 x nb 2
constexpr int kPackW3 = 10;                 // kb 4 x nb 1 (column 0 = w3)
constexpr int kPackW2T = 14;                // kb 4 x nb 2 (W2 transposed)
constexpr int kPackBlocks = 22;

__device__ __forceinline__ int c_row(int r, int lane) {
  return ((r >> 2) << 3) + ((lane >> 5) << 2) + (r & 3);
}
__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// GELU in its tanh form (Hendrycks and Gimpel, 2016), the tanh from one
// exponential and one hardware reciprocal (v_rcp_f32, 1 ulp; the GELUs feed
// BF16 operands): tanh(u) = 1 - 2 / (1 + e^{2u}) (e^{2u} overflowing to inf
// gives 1, underflowing to 0 gives -1)
__device__ __forceinline__ float gelu_tanh_arg(float z) {
  return 0.7978845608028654f * (z + 0.044715f * z * z * z);
}
__device__ __forceinline__ float fast_tanh(float u) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * u));
}
__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + fast_tanh(gelu_tanh_arg(z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const float t = fast_tanh(gelu_tanh_arg(z));
  return 0.5f * (1.0f + t) +
         0.5f * z * (1.0f - t * t) * 0.7978845608028654f * (1.0f + 0.134145f * z * z);
}
__device__ __forceinline__ float bf(float x) { return (float)(__bf16)x; }

// ---------------------------------------------------------------------------
// features: G lanes per node (8 for degree <= kFinGroupMax, 32 for degree <=
// kFinHalfMax, 64 up to kFinBlockMin), one workgroup per hub
// ---------------------------------------------------------------------------
// Moments of the cluster degrees. Per arc (s, a), with c = k_s + k_a - 4,
// the clusters through a have degree c + k_b for the n = k_s + k_a - 2
// nodes b in N(s) \ {a} (stars) and N(a) \ {s} (paths), so with P_j the
// sum of k_b^j over those b (from the sums of both nodes' neighbour degrees
// to the power j, less k_a^j and k_s^j),
//   sum d^2 = n c^2 + 2 c P_1 + P_2
//   sum d^3 = n c^3 + 3 c^2 P_1 + 3 c P_2 + P_3
//   sum d^4 = n c^4 + 4 c^3 P_1 + 6 c^2 P_2 + 4 c P_3 + P_4
// (triangle clusters taken without their -2). With x = d / mean - 1 over the
// node's event sequences, ln N - EF = E[(1 + x) ln(1 + x)]
// = m2 / 2 - m3 / 6 + m4 / 12 - ..., m_j = E[x^j]; the features carry m2,
// m3 and m4. No triangle pass is needed.
struct FeatAcc {  // POD (lives in LDS); start from feat_zero()
  int64_t B, Q, c1;
  float mx, mn;
  double s1, s2, e2, e3, e4;
  __device__ void add(int2 ad, const NbrMoments &t, int64_t k, const NbrMoments &own) {
    const int64_t ka = ad.y;
    B += ka * ka;
    Q += t.s1;
    c1 += ka == 1;
    const float lk = logf((float)ka);
    mx = fmaxf(mx, lk);
    mn = fminf(mn, lk);
    s1 += lk;
    s2 += (double)lk * lk;
    const double n = (double)(k + ka - 2), c = (double)(k + ka - 4);
    const double dk = (double)k, da = (double)ka, dk2 = dk * dk, da2 = da * da;
    const double p1 = (double)(own.s1 - ka + t.s1 - k);
    const double p2 = (double)(own.s2 - ka * ka + t.s2 - k * k);
    const double p3 = own.s3 - da2 * da + t.s3 - dk2 * dk;
    const double p4 = own.s4 - da2 * da2 + t.s4 - dk2 * dk2;
    const double c2 = c * c;
    e2 += n * c2 + 2.0 * c * p1 + p2;
    e3 += n * c2 * c + 3.0 * c2 * p1 + 3.0 * c * p2 + p3;
    e4 += n * c2 * c2 + 4.0 * c2 * c * p1 + 6.0 * c2 * p2 + 4.0 * c * p3 + p4;
  }
  __device__ void merge(const FeatAcc &o) {
    B += o.B;
    Q += o.Q;
    c1 += o.c1;
    mx = fmaxf(mx, o.mx);
    mn = fminf(mn, o.mn);
    s1 += o.s1;
    s2 += o.s2;
    e2 += o.e2;
    e3 += o.e3;
    e4 += o.e4;
  }
};

__device__ __forceinline__ FeatAcc feat_zero() {
  FeatAcc a;
  a.B = a.Q = a.c1 = 0;
  a.mx = -1e30f;
  a.mn = 1e30f;
  a.s1 = a.s2 = a.e2 = a.e3 = a.e4 = 0.0;
  return a;
}

template <int G> __device__ __forceinline__ FeatAcc feat_reduce(FeatAcc a) {
  for (int off = G / 2; off > 0; off >>= 1) {
    FeatAcc o = feat_zero();
    o.B = __shfl_xor(a.B, off, G);
    o.Q = __shfl_xor(a.Q, off, G);
    o.c1 = __shfl_xor(a.c1, off, G);
    o.mx = __shfl_xor(a.mx, off, G);
    o.mn = __shfl_xor(a.mn, off, G);
    o.s1 = __shfl_xor(a.s1, off, G);
    o.s2 = __shfl_xor(a.s2, off, G);
    o.e2 = __shfl_xor(a.e2, off, G);
    o.e3 = __shfl_xor(a.e3, off, G);
    o.e4 = __shfl_xor(a.e4, off, G);
    a.merge(o);
  }
  return a;
}

// arcs first, first + stride, ... of node v (degree k, own sums own)
__device__ __forceinline__ void feat_arcs(const int2 *__restrict__ adj2,
                                          const NbrMoments *__restrict__ nbm, int32_t k,
                                          int32_t base, const NbrMoments &own, int32_t first,
                                          int32_t stride, FeatAcc &f) {
  for (int32_t e = base + first; e < base + k; e += stride) {
    const int2 ad = adj2[e];
    f.add(ad, nbm[ad.x], k, own);
  }
}

__device__ void feat_store(int32_t v, int32_t k, int64_t A, FeatAcc a,
                           const float *__restrict__ mean, const float *__restrict__ inv_std,
                           float *__restrict__ X, float *__restrict__ lnN) {
  const int64_t kk = k, B = a.B, Q = a.Q;
  const int64_t Ns = kk * kk - 2 * kk + A;
  // D without the triangle term
  const int64_t Ds = kk * (kk - 1) * (kk - 4) + 2 * (kk - 1) * A + (kk - 4) * (A - kk) +
                     (B - A) + (Q - kk * kk);
  // raw moments of d / mean, then the central moments of x = d / mean - 1
  double m2 = 0.0, m3 = 0.0, m4 = 0.0;
  if (Ns > 0 && Ds > 0) {
    const double q = (double)Ns / (double)Ds;  // 1 / mean
    const double r2 = a.e2 * q * q / (double)Ns, r3 = a.e3 * q * q * q / (double)Ns,
                 r4 = a.e4 * q * q * q * q / (double)Ns;
    m2 = r2 - 1.0;
    m3 = r3 - 3.0 * r2 + 2.0;
    m4 = r4 - 4.0 * r3 + 6.0 * r2 - 3.0;
  }
  float f[kF];
  f[0] = logf(1.0f + (float)kk);
  f[1] = logf(1.0f + (float)A);
  f[2] = logf(1.0f + (float)B);
  f[3] = (float)asinh(m3);
  f[4] = (float)asinh(m4);
  f[5] = logf(1.0f + (float)(A - kk));
  f[6] = logf(1.0f + (float)Ns);
  f[7] = logf(1.0f + (float)Ds);
  f[8] = (Ns > 0 && Ds > 0) ? (float)log((double)Ds / (double)Ns) : 0.0f;
  const double mean_lk = k > 0 ? a.s1 / k : 0.0;
  f[9] = k > 0 ? a.mx : 0.0f;
  f[10] = k > 0 ? a.mn : 0.0f;
  f[11] = (float)mean_lk;
  f[12] = k > 0 ? (float)sqrt(fmax(a.s2 / k - mean_lk * mean_lk, 0.0)) : 0.0f;
  f[13] = logf(1.0f + (float)Q);
  f[14] = k > 0 ? (float)a.c1 / (float)k : 0.0f;
  f[15] = (float)log1p(fmax(m2, 0.0));
  float *dst = X + (int64_t)v * kF;
#pragma unroll
  for (int i = 0; i < kF; ++i) dst[i] = mean ? (f[i] - mean[i]) * inv_std[i] : f[i];
  lnN[v] = Ns > 0 ? logf((float)Ns) : 0.0f;
}

// nodes == nullptr: nodes 0..count-1 of degree <= kmax; else the listed nodes
template <int G>
__global__ __launch_bounds__(256) void k_features(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ deg,
    const int2 *__restrict__ adj2, const NbrMoments *__restrict__ nbm,
    const int32_t *__restrict__ nodes, int64_t count, int32_t kmax,
    const float *__restrict__ mean, const float *__restrict__ inv_std, float *__restrict__ X,
    float *__restrict__ lnN) {
  const int sub = threadIdx.x & (G - 1);
  const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
  const int64_t rounds = (count + ngrp - 1) / ngrp;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t it = r * ngrp + grp;
    int32_t v = -1, k = 0;
    if (it < count) {
      v = nodes ? nodes[it] : (int32_t)it;
      k = deg[v];
      if (!nodes && k > kmax) v = -1;
    }
    if (v < 0) k = 0;
    FeatAcc f = feat_zero();
    NbrMoments own{0, 0, 0.0, 0.0};
    if (v >= 0) {
      own = nbm[v];
      feat_arcs(adj2, nbm, k, row_ptr[v], own, sub, G, f);
    }
    f = feat_reduce<G>(f);
    if (v >= 0 && sub == 0) feat_store(v, k, own.s1, f, mean, inv_std, X, lnN);
  }
}

__global__ __launch_bounds__(1024) void k_features_hub(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ deg,
    const int2 *__restrict__ adj2, const NbrMoments *__restrict__ nbm,
    const int32_t *__restrict__ nodes, int64_t count, const float *__restrict__ mean,
    const float *__restrict__ inv_std, float *__restrict__ X, float *__restrict__ lnN) {
  __shared__ FeatAcc sh[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int32_t v = nodes[it];
    const int32_t k = deg[v];
    FeatAcc f = feat_zero();
    const NbrMoments own = nbm[v];
    feat_arcs(adj2, nbm, k, row_ptr[v], own, tid, 1024, f);
    f = feat_reduce<64>(f);
    if (lane == 0) sh[wv] = f;
    __syncthreads();
    if (tid == 0) {
      FeatAcc a = sh[0];
      for (int w = 1; w < 16; ++w) a.merge(sh[w]);
      feat_store(v, k, own.s1, a, mean, inv_std, X, lnN);
    }
    __syncthreads();
  }
}

hipError_t launch_features(const Graph &g, const float *mean, const float *inv_std, float *X,
                           float *lnN, hipStream_t st) {
  auto cap = [](int64_t b, int64_t c) { return (unsigned)std::max<int64_t>(1, std::min(b, c)); };
  const int64_t n_wave = g.n_fin - g.n_fin_hub - g.n_fin_half;
  const int32_t *l_wave = g.fin_list + g.n_fin_hub, *l_half = l_wave + n_wave;
  if (g.n_fin_hub > 0)
    hipLaunchKernelGGL(k_features_hub, dim3(cap(g.n_fin_hub, 1 << 16)), dim3(1024), 0, st,
                       g.row_ptr, g.deg, g.adj2, g.nbm, g.fin_list, g.n_fin_hub, mean, inv_std, X,
                       lnN);
  hipLaunchKernelGGL(k_features<8>, dim3(cap(((int64_t)g.n * 8 + 255) / 256, 1 << 20)), dim3(256),
                     0, st, g.row_ptr, g.deg, g.adj2, g.nbm, nullptr, (int64_t)g.n, kFinGroupMax,
                     mean, inv_std, X, lnN);
  if (n_wave > 0)
    hipLaunchKernelGGL(k_features<64>, dim3(cap((n_wave * 64 + 255) / 256, 1 << 20)), dim3(256),
                       0, st, g.row_ptr, g.deg, g.adj2, g.nbm, l_wave, n_wave, 0, mean, inv_std,
                       X, lnN);
  if (g.n_fin_half > 0)
    hipLaunchKernelGGL(k_features<32>, dim3(cap((g.n_fin_half * 32 + 255) / 256, 1 << 20)),
                       dim3(256), 0, st, g.row_ptr, g.deg, g.adj2, g.nbm, l_half, g.n_fin_half, 0,
                       mean, inv_std, X, lnN);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MLP on one 32-row tile per wavefront
// ---------------------------------------------------------------------------
struct TileLds {
  __bf16 x[32][kF];
  __bf16 h1[32][kH];
  __bf16 h2[32][kH];
  __bf16 dz[32][kH];
  float dy[32];
};

__device__ __forceinline__ bf16x8 lds_a(const __bf16 *rowmajor, int ld, int kb) {
  // A fragment: row lane % 32, columns 16 kb + 8 (lane / 32) .. + 7
  const int lane = threadIdx.x & 63;
  return *reinterpret_cast<const bf16x8 *>(rowmajor + (lane & 31) * ld + kb * 16 +
                                           ((lane >> 5) << 3));
}
// B fragment from a row-major [K][ld] LDS matrix: column nb*32 + lane%32,
// rows 16 kb + 8 (lane / 32) .. + 7
__device__ __forceinline__ bf16x8 lds_b(const __bf16 *rowmajor, int ld, int kb, int nb) {
  const int lane = threadIdx.x & 63;
  bf16x8 v;
  const int r0 = kb * 16 + ((lane >> 5) << 3), c = nb * 32 + (lane & 31);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = rowmajor[(r0 + j) * ld + c];
  return v;
}
// A fragment of the transpose of a row-major [K][ld] LDS matrix: A[m][kk] =
// M[kk][m], m = mb*32 + lane%32 (zero when m >= mlim), kk = 16 kb + 8 (lane/32) + j
__device__ __forceinline__ bf16x8 lds_at(const __bf16 *rowmajor, int ld, int kb, int mb,
                                         int mlim) {
  const int lane = threadIdx.x & 63;
  bf16x8 v;
  const int r0 = kb * 16 + ((lane >> 5) << 3), m = mb * 32 + (lane & 31);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = m < mlim ? rowmajor[(r0 + j) * ld + m] : (__bf16)0.0f;
  return v;
}
__device__ __forceinline__ bf16x8 wpack(const __bf16 *pack, int block) {
  return reinterpret_cast<const bf16x8 *>(pack)[block * 64 + (threadIdx.x & 63)];
}

// Forward of one tile. Rows r0 .. r0+31 of X (row index through `perm` when
// given); rows at or past `rows` are zero. Leaves z1, z2 (pre-activations,
// C layout) in registers and x, h1, h2 (bf16) in LDS; returns y for the rows
// held by lanes 0 and 32 (C layout of column 0) in yv.
__device__ void tile_forward(const float *__restrict__ X, const int32_t *__restrict__ perm,
                             int64_t r0, int64_t rows, const float *__restrict__ P,
                             const __bf16 *__restrict__ pack, TileLds &t, f32x16 z1[2],
                             f32x16 z2[2], f32x16 &yv) {
  const int lane = threadIdx.x & 63;
  {
    const int i = lane & 31, c0 = (lane >> 5) * 8;
    const int64_t row = r0 + i;
    float xv[8];
    if (row < rows) {
      const int64_t src = perm ? perm[row] : row;
      const float4 a = *reinterpret_cast<const float4 *>(X + src * kF + c0);
      const float4 b = *reinterpret_cast<const float4 *>(X + src * kF + c0 + 4);
      xv[0] = a.x; xv[1] = a.y; xv[2] = a.z; xv[3] = a.w;
      xv[4] = b.x; xv[5] = b.y; xv[6] = b.z; xv[7] = b.w;
    } else {
      for (int j = 0; j < 8; ++j) xv[j] = 0.0f;
    }
    for (int j = 0; j < 8; ++j) t.x[i][c0 + j] = (__bf16)xv[j];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  const bf16x8 ax = lds_a(&t.x[0][0], kF, 0);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    f32x16 c = {};
    c = mfma(ax, wpack(pack, kPackW1 + nb), c);
    const float b1 = P[kOffB1 + nb * 32 + (lane & 31)];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      c[r] += b1;
      t.h1[c_row(r, lane)][nb * 32 + (lane & 31)] = (__bf16)gelu(c[r]);
    }
    z1[nb] = c;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    f32x16 c = {};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      c = mfma(lds_a(&t.h1[0][0], kH, kb), wpack(pack, kPackW2 + kb * 2 + nb), c);
    const float b2 = P[kOffB2 + nb * 32 + (lane & 31)];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      c[r] += b2;
      t.h2[c_row(r, lane)][nb * 32 + (lane & 31)] = (__bf16)gelu(c[r]);
    }
    z2[nb] = c;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  f32x16 c = {};
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) c = mfma(lds_a(&t.h2[0][0], kH, kb), wpack(pack, kPackW3 + kb), c);
  const float b3 = P[kOffB3];
#pragma unroll
  for (int r = 0; r < 16; ++r) c[r] += b3;
  yv = c;
}

// inference: y for rows [0, rows); out_ef = max(0, lnN - y) when lnN given
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ X, int64_t rows,
                                                     const float *__restrict__ P,
                                                     const __bf16 *__restrict__ pack,
                                                     const float *__restrict__ lnN,
                                                     float *__restrict__ y_out,
                                                     double *__restrict__ ef_out) {
  __shared__ TileLds tl[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t tiles = (rows + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < tiles; tile += (int64_t)gridDim.x * 4) {
    f32x16 z1[2], z2[2], yv;
    tile_forward(X, nullptr, tile * 32, rows, P, pack, tl[wv], z1, z2, yv);
    if ((lane & 31) == 0) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = tile * 32 + c_row(r, lane);
        if (row < rows) {
          if (y_out) y_out[row] = yv[r];
          if (ef_out) {
            const float e = lnN[row] - yv[r];
            ef_out[row] = e > 0.0f ? (double)e : 0.0;
          }
        }
      }
    }
  }
}

// Training: gradients of the mean squared error over the rows perm[b0 .. b0+nb)
// (scale = 2 / nb), accumulated per wavefront into part[wave][kParams]; the
// squared-error sum per wavefront into part_loss[wave].
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ X,
                                                  const float *__restrict__ Yt,
                                                  const int32_t *__restrict__ perm, int64_t b0,
                                                  int64_t nrows, const float *__restrict__ P,
                                                  const __bf16 *__restrict__ pack,
                                                  float *__restrict__ part,
                                                  float *__restrict__ part_loss) {
  __shared__ TileLds tl[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  TileLds &t = tl[wv];
  const int64_t wave = (int64_t)blockIdx.x * 4 + wv;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const int64_t tiles = (nrows + 31) / 32;
  const float scale = 2.0f / (float)nrows;
  const int col = lane & 31;
  f32x16 gW2[2][2] = {}, gW1[2] = {};
  float gb1[2] = {0.f, 0.f}, gb2[2] = {0.f, 0.f}, gw3[2] = {0.f, 0.f}, gb3 = 0.f, lsum = 0.f;
  float w3b[2];
  for (int nb = 0; nb < 2; ++nb) w3b[nb] = bf(P[kOffW3 + nb * 32 + col]);
  const int32_t *pr = perm + b0;
  for (int64_t tile = wave; tile < tiles; tile += nwaves) {
    f32x16 z1[2], z2[2], yv;
    tile_forward(X, pr, tile * 32, nrows, P, pack, t, z1, z2, yv);
    if (col == 0) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = c_row(r, lane);
        const int64_t row = tile * 32 + i;
        float d = 0.f;
        if (row < nrows) {
          const float res = yv[r] - Yt[pr[row]];
          lsum += res * res;
          d = scale * res;
        }
        t.dy[i] = d;
        gb3 += d;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // layer 3 and dz2 = dy w3 * gelu'(z2)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = c_row(r, lane);
        const float d = t.dy[i];
        gw3[nb] += (float)t.h2[i][nb * 32 + col] * d;
        const float dz = d * w3b[nb] * gelu_grad(z2[nb][r]);
        gb2[nb] += dz;
        t.dz[i][nb * 32 + col] = (__bf16)dz;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // dW2 += h1^T dz2 ; dh1 = dz2 W2^T
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const bf16x8 a = lds_at(&t.h1[0][0], kH, kb, mb, kH);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) gW2[mb][nb] = mfma(a, lds_b(&t.dz[0][0], kH, kb, nb), gW2[mb][nb]);
      }
    }
    f32x16 dh1[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      f32x16 c = {};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        c = mfma(lds_a(&t.dz[0][0], kH, kb), wpack(pack, kPackW2T + kb * 2 + nb), c);
      dh1[nb] = c;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // dz1 = dh1 * gelu'(z1)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dz = dh1[nb][r] * gelu_grad(z1[nb][r]);
        gb1[nb] += dz;
        t.dz[c_row(r, lane)][nb * 32 + col] = (__bf16)dz;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // dW1 += x^T dz1 (rows 16..31 of the A operand are zero)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const bf16x8 a = lds_at(&t.x[0][0], kF, kb, 0, kF);
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) gW1[nb] = mfma(a, lds_b(&t.dz[0][0], kH, kb, nb), gW1[nb]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  // write this wavefront's partial gradient
  float *g = part + wave * kParams;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = c_row(r, lane);
      if (m < kF) g[kOffW1 + m * kH + nb * 32 + col] = gW1[nb][r];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) g[kOffW2 + (mb * 32 + m) * kH + nb * 32 + col] = gW2[mb][nb][r];
    }
    const float b1 = gb1[nb] + __shfl_xor(gb1[nb], 32, 64);
    const float b2 = gb2[nb] + __shfl_xor(gb2[nb], 32, 64);
    const float w3 = gw3[nb] + __shfl_xor(gw3[nb], 32, 64);
    if (lane < 32) {
      g[kOffB1 + nb * 32 + col] = b1;
      g[kOffB2 + nb * 32 + col] = b2;
      g[kOffW3 + nb * 32 + col] = w3;
    }
  }
  const float b3 = gb3 + __shfl_xor(gb3, 32, 64);
  const float ls = lsum + __shfl_xor(lsum, 32, 64);
  if (lane == 0) {
    g[kOffB3] = b3;
    part_loss[wave] = ls;
  }
}

// grad[p] = sum over wavefronts (fixed order); loss = sum of part_loss
__global__ void k_grad_reduce(const float *__restrict__ part, const float *__restrict__ part_loss,
                              int32_t nwaves, float *__restrict__ grad, float *__restrict__ loss) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= kParams; p += gridDim.x * blockDim.x) {
    if (p < kParams) {
      double s = 0.0;
      for (int w = 0; w < nwaves; ++w) s += part[(int64_t)w * kParams + p];
      grad[p] = (float)s;
    } else {
      double s = 0.0;
      for (int w = 0; w < nwaves; ++w) s += part_loss[w];
      *loss = (float)s;
    }
  }
}

// Re-pack the BF16 B-operand blocks from the FP32 masters.
__global__ void k_pack(const float *__restrict__ P, __bf16 *__restrict__ pack) {
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < kPackBlocks * 64 * 8;
       idx += gridDim.x * blockDim.x) {
    const int block = idx / 512, lane = (idx / 8) % 64, j = idx % 8;
    const int kin = (lane >> 5) * 8 + j, n = lane & 31;
    float v = 0.f;
    if (block < kPackW2) {  // W1: kb 0, nb = block
      v = P[kOffW1 + kin * kH + block * 32 + n];
    } else if (block < kPackW3) {  // W2: (kb, nb)
      const int b = block - kPackW2, kb = b / 2, nb = b % 2;
      v = P[kOffW2 + (kb * 16 + kin) * kH + nb * 32 + n];
    } else if (block < kPackW2T) {  // w3 as column 0
      const int kb = block - kPackW3;
      v = n == 0 ? P[kOffW3 + kb * 16 + kin] : 0.f;
    } else {  // W2^T: B[k][n] = W2[n][k]
      const int b = block - kPackW2T, kb = b / 2, nb = b % 2;
      v = P[kOffW2 + (nb * 32 + n) * kH + kb * 16 + kin];
    }
    pack[idx] = (__bf16)v;
  }
}

// Adam (Kingma and Ba, 2015) on the FP32 masters: step t (1-based)
__global__ void k_adam(float *__restrict__ P, float *__restrict__ M, float *__restrict__ V,
                       const float *__restrict__ grad, float lr, float b1, float b2, float eps,
                       float wd, int32_t t) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < kParams; p += gridDim.x * blockDim.x) {
    const float g = grad[p];
    const float m = b1 * M[p] + (1.0f - b1) * g;
    const float v = b2 * V[p] + (1.0f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    P[p] -= lr * ((m / c1) / (sqrtf(v / c2) + eps) + wd * P[p]);
  }
}

hipError_t launch_mlp_pack(const float *P, __bf16 *pack, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(22), dim3(512), 0, st, P, pack);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *X, int64_t rows, const float *P, const __bf16 *pack,
                              const float *lnN, float *y, double *ef, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int64_t tiles = (rows + 31) / 32;
  const unsigned blocks = (unsigned)std::min<int64_t>((tiles + 3) / 4, 1 << 16);
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, st, X, rows, P, pack, lnN, y, ef);
  return hipGetLastError();
}

// gradient of the mean squared error over perm[b0 .. b0+nrows) with `nblocks`
// workgroups of 4 wavefronts; part has room for nblocks*4 partials
hipError_t launch_mlp_grad(const float *X, const float *Yt, const int32_t *perm, int64_t b0,
                           int64_t nrows, const float *P, const __bf16 *pack, float *part,
                           float *part_loss, int32_t nblocks, float *grad, float *loss,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblocks), dim3(256), 0, st, X, Yt, perm, b0, nrows, P, pack,
                     part, part_loss);
  hipLaunchKernelGGL(k_grad_reduce, dim3((kParams + 256) / 256), dim3(256), 0, st, part,
                     part_loss, nblocks * 4, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float *P, float *M, float *V, const float *grad, float lr, float b1,
                       float b2, float eps, float wd, int32_t t, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, P, M, V, grad, lr, b1,
                     b2, eps, wd, t);
  return hipGetLastError();
}

int32_t mlp_param_count() { return kParams; }
int32_t mlp_pack_count() { return kPackBlocks * 64 * 8; }

}  // namespace efi
