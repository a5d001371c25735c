// Host test driver for the library's CSR checks, built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py: every array
// is a heap block of exactly its stated length, so a read past any of them
// stops the run. Prints "ok" and exits 0 when every case returns its expected
// status.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "csr_check.h"

using efi::csr_check_bounds;
using efi::csr_validate;

static int failures = 0;

static ef_status run(bool full, int32_t n, const std::vector<int32_t> &rp,
                     const std::vector<int32_t> &ci, int64_t nnz) {
  // exact-size copies (no slack for an overread to land in)
  int32_t *r = rp.empty() ? nullptr : new int32_t[rp.size()];
  int32_t *c = ci.empty() ? nullptr : new int32_t[ci.size()];
  if (r) std::memcpy(r, rp.data(), sizeof(int32_t) * rp.size());
  if (c) std::memcpy(c, ci.data(), sizeof(int32_t) * ci.size());
  char msg[256];
  const ef_status s = full ? csr_validate(n, nnz, r, c, msg, sizeof(msg))
                           : csr_check_bounds(n, nnz, r, c, msg, sizeof(msg));
  delete[] r;
  delete[] c;
  return s;
}

static void expect(const char *name, bool full, int32_t n, std::vector<int32_t> rp,
                   std::vector<int32_t> ci, ef_status want) {
  const ef_status got = run(full, n, rp, ci, (int64_t)ci.size());
  if (got != want) {
    std::printf("FAIL %s (%s): got %d want %d\n", name, full ? "validate" : "bounds", got, want);
    ++failures;
  }
}

static uint64_t lcg(uint64_t &x) {
  x = x * 6364136223846793005ull + 1442695040888963407ull;
  return x >> 33;
}

int main() {
  // path 0-1-2 plus isolated node 3
  expect("valid", true, 4, {0, 1, 3, 4, 4}, {1, 0, 2, 1}, EF_OK);
  expect("valid", false, 4, {0, 1, 3, 4, 4}, {1, 0, 2, 1}, EF_OK);
  expect("empty", true, 0, {0}, {}, EF_OK);
  expect("isolated", true, 3, {0, 0, 0, 0}, {}, EF_OK);
  expect("self_loop", true, 3, {0, 2, 3, 4}, {0, 1, 0, 1}, EF_ERR_SELF_LOOP);
  expect("duplicate", true, 2, {0, 2, 4}, {1, 1, 0, 0}, EF_ERR_DUPLICATE);
  expect("unsorted", true, 3, {0, 2, 3, 4}, {2, 1, 0, 0}, EF_ERR_UNSORTED);
  expect("not_symmetric", true, 3, {0, 1, 1, 1}, {1}, EF_ERR_NOT_SYMMETRIC);
  for (bool full : {true, false}) {
    expect("row_ptr_decreasing", full, 3, {0, 2, 1, 2}, {1, 2}, EF_ERR_UNSORTED);
    expect("offset_past_end", full, 3, {0, 9, 1, 2}, {1, 2}, EF_ERR_UNSORTED);
    expect("negative_offset", full, 3, {0, -5, 1, 2}, {1, 2}, EF_ERR_UNSORTED);
    expect("out_of_range", full, 2, {0, 1, 2}, {1, 5}, EF_ERR_RANGE);
    expect("negative_id", full, 2, {0, 1, 2}, {1, -1}, EF_ERR_RANGE);
    expect("row_ptr_start", full, 2, {1, 2, 3}, {1, 0}, EF_ERR_RANGE);
    expect("row_ptr_end", full, 2, {0, 1, 1}, {1, 0}, EF_ERR_RANGE);
  }
  // random garbage CSRs: whatever the status, no read may leave the arrays
  uint64_t x = 12345;
  int accepted = 0;
  for (int it = 0; it < 20000; ++it) {
    const int32_t n = (int32_t)(lcg(x) % 9);
    const int32_t m = (int32_t)(lcg(x) % 12);
    std::vector<int32_t> rp((size_t)n + 1), ci((size_t)m);
    const int mode = (int)(lcg(x) % 3);
    for (auto &v : rp) v = (int32_t)(lcg(x) % (m + 2)) - (mode == 0 ? 1 : 0);
    if (mode != 0) {
      rp[0] = 0;
      rp[n] = m;
    }
    if (mode == 2)
      for (int32_t v = 1; v <= n; ++v) rp[v] = rp[v] < rp[v - 1] ? rp[v - 1] : rp[v];
    for (auto &v : ci) v = (int32_t)(lcg(x) % (n + 2)) - 1;
    const bool full = lcg(x) & 1;
    const ef_status s = run(full, n, rp, ci, m);
    if (s == EF_OK) ++accepted;
    if (s != EF_OK && s != EF_ERR_RANGE && s != EF_ERR_UNSORTED && s != EF_ERR_DUPLICATE &&
        s != EF_ERR_SELF_LOOP && s != EF_ERR_NOT_SYMMETRIC) {
      std::printf("FAIL fuzz %d: status %d\n", it, s);
      ++failures;
    }
  }
  if (failures) return 1;
  std::printf("ok (%d random CSRs accepted)\n", accepted);
  return 0;
}
