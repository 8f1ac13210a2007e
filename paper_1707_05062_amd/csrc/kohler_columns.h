// Column arithmetic of the curve kernel's row loads (kohler_kernels.hip), kept free of HIP so that a
// CPU test can check, for every width, that each column a lane reads lies inside the row. Strip s of
// a row covers the columns [s * SW, (s + 1) * SW) with SW = 64 * K; lane l's first column is
// c = s * SW + l * K. Not installed.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define KOHLER_HD __host__ __device__
#else
#define KOHLER_HD
#endif

namespace kohler {

// A column exists right of the strip: every lane's K pixels and its right neighbour are inside.
KOHLER_HD inline bool strip_full(int64_t s, int sw, int64_t W) { return (s + 1) * sw < W; }
// The strip ends at or before the right border (the 8-bit packed path; at the border the right
// neighbour read is the row's last pixel).
KOHLER_HD inline bool strip_inside(int64_t s, int sw, int64_t W) { return (s + 1) * sw <= W; }
// First column of a packed load of K pixels: lanes past the row end of the last strip re-read the
// row's last aligned chunk (used only when W is a multiple of K).
KOHLER_HD inline int64_t packed_column(int64_t c, int K, int64_t W, bool full) {
    return full ? c : (c < W - K ? c : W - K);
}
// Column of pixel k of an element load: clamped to the row's last pixel.
KOHLER_HD inline int64_t element_column(int64_t c, int k, int64_t W, bool full) {
    return full ? c + k : (c + k < W - 1 ? c + k : W - 1);
}
// The pixel right of strip s (clamped to the row's last pixel) and left of it (clamped to 0).
KOHLER_HD inline int64_t right_edge_column(int64_t s, int sw, int64_t W) {
    return (s + 1) * sw < W - 1 ? (s + 1) * sw : W - 1;
}
KOHLER_HD inline int64_t left_edge_column(int64_t s, int sw) { return s * sw > 0 ? s * sw - 1 : 0; }

// How strip s of a row is loaded (strip_range): the 8-bit packed path (instances that have it,
// aligned rows, strips inside the row), full strips with vector or element loads, and the last
// strip with vector loads (W a multiple of K) or clamped element loads.
enum StripPath { PATH_PK = 0, PATH_FULL_PACKED, PATH_FULL_ELEM, PATH_LAST_PACKED, PATH_LAST_ELEM };
KOHLER_HD inline StripPath strip_path(int64_t s, int K, int64_t W, bool vec_ok, bool has_pk) {
    const int sw = 64 * K;
    if (has_pk && vec_ok && strip_inside(s, sw, W)) return PATH_PK;
    if (strip_full(s, sw, W)) return vec_ok ? PATH_FULL_PACKED : PATH_FULL_ELEM;
    return (vec_ok && W % K == 0) ? PATH_LAST_PACKED : PATH_LAST_ELEM;
}

}  // namespace kohler
