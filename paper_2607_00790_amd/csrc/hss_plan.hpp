// Host-side planning rules of the HSS build that depend only on sizes.
#pragma once

#include <cstdint>

namespace bm {
namespace hss {

// Work guard of the ID.  A box whose stacked near/proxy matrix M_b (candidate
// rows x active unknowns, complex FP64) would exceed kMaxIdEntries entries, or
// a body whose boxes' matrices would exceed kMaxLevelIdEntries together, is
// not compressed further: its current boxes' skeletons form its dense root.
// The column-pivoted QR of such a matrix moves it through memory once per
// elimination step (tens of thousands of steps at these sizes), and the
// matrix alone would fill a large part of device memory; the dense root it
// avoids is a few large products on the matrix cores instead.  One box of
// 19096 unknowns against 62236 rows (1.2e9 entries) is the case this stops.
constexpr int64_t kMaxIdEntries = int64_t{1} << 26;        // 1 GiB per box
constexpr int64_t kMaxLevelIdEntries = int64_t{1} << 31;   // 32 GiB per body and level

inline bool id_box_over_budget(int64_t rows, int64_t unknowns) {
    return rows > 0 && unknowns > 0 && rows > kMaxIdEntries / unknowns;
}

// total: the sum of rows x unknowns over the body's boxes at this level
inline bool id_level_over_budget(int64_t total) { return total > kMaxLevelIdEntries; }

}  // namespace hss
}  // namespace bm
