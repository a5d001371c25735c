// Host-side checks of an int32 CSR graph (no device code, no HIP headers), so
// that they can also be built on their own with host sanitizers.
#pragma once

#include <cstddef>
#include <cstdint>

#include "ef.h"

namespace efi {

// The full check behind ef_validate_csr: the CSR is the simple undirected
// graph that Algorithm 1 takes (offsets from 0 to nnz, non-decreasing; ids in
// range; rows strictly ascending, so no duplicates; no self-loops; every arc
// has its reverse). Returns the first violation; msg (cap bytes) names it.
ef_status csr_validate(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                       char *msg, size_t cap);

// The O(n + nnz) part that makes the arrays safe to index: row_ptr[0] == 0,
// row_ptr non-decreasing, row_ptr[n] == nnz, every neighbour id in [0, n).
// col_idx may be null (the column range is then left to the caller).
ef_status csr_check_bounds(int32_t n, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col_idx, char *msg, size_t cap);

}  // namespace efi
