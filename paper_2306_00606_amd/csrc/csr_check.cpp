// Host-side CSR checks (see csr_check.h).
#include "csr_check.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>

namespace efi {

static ef_status fail(ef_status s, char *msg, size_t cap, const char *fmt, ...) {
  if (msg && cap) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, cap, fmt, ap);
    va_end(ap);
  }
  return s;
}

ef_status csr_check_bounds(int32_t n, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col_idx, char *msg, size_t cap) {
  if (n < 0 || nnz < 0)
    return fail(EF_ERR_ARG, msg, cap, "negative size (n=%d, nnz=%lld)", n, (long long)nnz);
  if (nnz >= (int64_t)INT32_MAX)
    return fail(EF_ERR_OVERFLOW, msg, cap, "nnz=%lld does not fit int32 offsets", (long long)nnz);
  if (!row_ptr) return fail(EF_ERR_ARG, msg, cap, "null row_ptr");
  if (row_ptr[0] != 0)
    return fail(EF_ERR_RANGE, msg, cap, "row_ptr[0] = %d, expected 0", row_ptr[0]);
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v])
      return fail(EF_ERR_UNSORTED, msg, cap, "row_ptr decreases at row %d", v);
  if ((int64_t)row_ptr[n] != nnz)
    return fail(EF_ERR_RANGE, msg, cap, "row_ptr[n] = %d but nnz = %lld", row_ptr[n],
                (long long)nnz);
  if (col_idx) {
    const uint32_t un = (uint32_t)n;
    for (int64_t e = 0; e < nnz; ++e)
      if ((uint32_t)col_idx[e] >= un) {
        // name the row: the last v with row_ptr[v] <= e
        const int32_t v = (int32_t)(std::upper_bound(row_ptr, row_ptr + n + 1, (int32_t)e) -
                                    row_ptr) - 1;
        return fail(EF_ERR_RANGE, msg, cap, "row %d: neighbour %d out of range [0, %d)", v,
                    col_idx[e], n);
      }
  }
  return EF_OK;
}

ef_status csr_validate(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                       char *msg, size_t cap) {
  if (n < 0 || nnz < 0)
    return fail(EF_ERR_ARG, msg, cap, "negative size (n=%d, nnz=%lld)", n, (long long)nnz);
  if (!row_ptr || (nnz > 0 && !col_idx)) return fail(EF_ERR_ARG, msg, cap, "null array");
  ef_status s = csr_check_bounds(n, nnz, row_ptr, col_idx, msg, cap);
  if (s != EF_OK) return s;
  for (int32_t v = 0; v < n; ++v) {
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int32_t x = col_idx[e];
      if (x == v) return fail(EF_ERR_SELF_LOOP, msg, cap, "row %d: self-loop", v);
      if (e > row_ptr[v]) {
        if (col_idx[e - 1] == x)
          return fail(EF_ERR_DUPLICATE, msg, cap, "row %d: neighbour %d listed twice", v, x);
        if (col_idx[e - 1] > x)
          return fail(EF_ERR_UNSORTED, msg, cap, "row %d: neighbours not ascending at position %d",
                      v, e - row_ptr[v]);
      }
    }
  }
  for (int32_t v = 0; v < n; ++v)
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int32_t x = col_idx[e];
      if (!std::binary_search(col_idx + row_ptr[x], col_idx + row_ptr[x + 1], v))
        return fail(EF_ERR_NOT_SYMMETRIC, msg, cap, "arc %d->%d has no reverse arc %d->%d", v, x,
                    x, v);
    }
  return EF_OK;
}

}  // namespace efi
