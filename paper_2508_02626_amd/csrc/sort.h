// Device-wide scan and stable radix sort (see sort.hip).
#pragma once
#include "common.h"

namespace fmm {
size_t scan_scratch_bytes(int64_t n);
// out[0..n]: exclusive prefix sums of in[0..n), out[n] = total
void scan_exclusive(const int64_t *in, int64_t *out, int64_t n, int64_t *scratch, hipStream_t s);
constexpr int kMaxScanBatch = 8;
size_t scan_multi_scratch_bytes(int64_t n, int count);
// count (<= kMaxScanBatch) scans of length n in one set of launches
void scan_exclusive_multi(const int64_t *const *in, int64_t *const *out, int count, int64_t n,
                          int64_t *scratch, hipStream_t s);
size_t sort_scratch_bytes(int n);
void radix_sort_pairs(uint64_t *keys, int32_t *vals, uint64_t *tk, int32_t *tv, int n, int bits,
                      int32_t *scratch, hipStream_t s);
} // namespace fmm
