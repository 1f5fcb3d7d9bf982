// Host-side planning of the HSS build: rules that depend only on sizes, and
// the boxes' proxy-circle geometry.
#pragma once

#include <algorithm>
#include <cmath>
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

// Level l of a body's tree (paper Sec. III, Fig. 2): its nodes [nlo, nlo + nn)
// split into 2^l boxes of consecutive nodes, box b holding
// [nlo + floor(b nn / 2^l), nlo + floor((b + 1) nn / 2^l)).  Per box: the
// centre (the mean of its nodes), the proxy circle's radius (proxy_ratio times
// the largest distance of a node from the centre) and its number of proxy
// points (P; with adapt, at least ceil(2 kmax r) + 32 so that the circle is
// sampled finely enough at the larger wavenumber; at most 2^20).  x, y: the
// node coordinates; box_c: x, y and radius per box; box_p: points per box.
inline void level_box_geometry(const double* x, const double* y, int64_t nlo, int64_t nn, int l,
                               double proxy_ratio, int64_t P, bool adapt, double kmax, double* box_c,
                               int32_t* box_p) {
    const int64_t nb = int64_t{1} << l;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t lo = nlo + ((b * nn) >> l), hi = nlo + (((b + 1) * nn) >> l);
        double cx = 0, cy = 0;
        for (int64_t i = lo; i < hi; ++i) {
            cx += x[i];
            cy += y[i];
        }
        cx /= static_cast<double>(hi - lo);
        cy /= static_cast<double>(hi - lo);
        double r2 = 0;
        for (int64_t i = lo; i < hi; ++i) r2 = std::max(r2, (x[i] - cx) * (x[i] - cx) + (y[i] - cy) * (y[i] - cy));
        const double rp = proxy_ratio * std::sqrt(r2);
        box_c[3 * b] = cx;
        box_c[3 * b + 1] = cy;
        box_c[3 * b + 2] = rp;
        int64_t pb = P;
        if (adapt) pb = std::max<int64_t>(P, static_cast<int64_t>(std::ceil(2.0 * kmax * rp)) + 32);
        box_p[b] = static_cast<int32_t>(std::min<int64_t>(pb, int64_t{1} << 20));
    }
}

}  // namespace hss
}  // namespace bm
