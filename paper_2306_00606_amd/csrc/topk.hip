// Top-k spreaders: the k nodes of largest Expected Force ("identification of
// key nodes", the paper's title and Sec. 1). Order: EF descending, ties by
// node id ascending.
//
// EF values are non-negative doubles, whose IEEE bit patterns order like the
// values as unsigned 64-bit integers. A stable descending radix sort of
// (bits, id) pairs with ids supplied in ascending order yields exactly that
// order; the first k pairs are the answer.
#include <hipcub/hipcub.hpp>

#include "ef_internal.h"

namespace efi {

__global__ void k_topk_keys(const double *__restrict__ ef, int32_t n,
                            unsigned long long *__restrict__ keys, int32_t *__restrict__ ids) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = ef[i];
    keys[i] = v > 0.0 ? (unsigned long long)__double_as_longlong(v) : 0ull;
    ids[i] = (int32_t)i;
  }
}

__global__ void k_topk_out(const unsigned long long *__restrict__ keys,
                           const int32_t *__restrict__ ids, int32_t k, int32_t *__restrict__ nodes,
                           double *__restrict__ ef) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
       i += (int64_t)gridDim.x * blockDim.x) {
    nodes[i] = ids[i];
    if (ef) ef[i] = __longlong_as_double((long long)keys[i]);
  }
}

size_t topk_scratch_bytes(int32_t n) {
  size_t temp = 0;
  (void)hipcub::DeviceRadixSort::SortPairsDescending(
      nullptr, temp, (const unsigned long long *)nullptr, (unsigned long long *)nullptr,
      (const int32_t *)nullptr, (int32_t *)nullptr, n);
  return temp + (size_t)n * (2 * sizeof(unsigned long long) + 2 * sizeof(int32_t)) + 1024;
}

hipError_t launch_topk(const double *ef, int32_t n, int32_t k, void *scratch,
                       size_t scratch_bytes, int32_t *nodes, double *ef_out, hipStream_t st) {
  if (n <= 0 || k <= 0) return hipSuccess;
  char *p = (char *)scratch;
  auto take = [&](size_t b) {
    char *r = p;
    p += (b + 255) & ~(size_t)255;
    return r;
  };
  auto *kin = (unsigned long long *)take(sizeof(unsigned long long) * (size_t)n);
  auto *kout = (unsigned long long *)take(sizeof(unsigned long long) * (size_t)n);
  auto *iin = (int32_t *)take(sizeof(int32_t) * (size_t)n);
  auto *iout = (int32_t *)take(sizeof(int32_t) * (size_t)n);
  size_t temp = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, temp, kin, kout, iin,
                                                              iout, n, 0, 64, st);
  if (e != hipSuccess) return e;
  void *tmp = take(temp);
  if ((size_t)(p - (char *)scratch) > scratch_bytes) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_topk_keys, dim3(blocks), dim3(256), 0, st, ef, n, kin, iin);
  e = hipcub::DeviceRadixSort::SortPairsDescending(tmp, temp, kin, kout, iin, iout, n, 0, 64, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_topk_out, dim3((unsigned)std::min<int64_t>((k + 255) / 256, 65536)),
                     dim3(256), 0, st, kout, iout, k, nodes, ef_out);
  return hipGetLastError();
}

}  // namespace efi
