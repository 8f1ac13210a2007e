// CPU test of the curve kernel's column arithmetic (paper_1707_05062_amd/csrc/kohler_columns.h): for
// every width up to a few strips, pixel size and pixels per lane, every column a lane reads on the
// path strip_path() picks lies inside the row [0, W): the pixels of a slot (packed loads as a whole
// K-pixel block), and the edge pixels right and left of the strip. Built with g++ under the address
// and undefined-behaviour sanitizers by tests/test_host_sanitizers.py.
#include <cstdio>
#include <initializer_list>

#include "kohler_columns.h"

using namespace kohler;

static long failures = 0, checked = 0;

static void inside(long long col, long long W, const char *what, long long s, int lane, int K, long long Wv) {
    ++checked;
    if (col < 0 || col >= W) {
        if (failures < 20) std::fprintf(stderr, "%s: column %lld outside [0, %lld) (strip %lld lane %d K %d W %lld)\n",
                                        what, col, W, s, lane, K, Wv);
        ++failures;
    }
}

int main() {
    for (int K : {4, 8}) {
        for (int esz : {1, 2}) {
            const bool has_pk = esz == 1 && K == 8;  // the 8-bit, 8-pixel instances of the banded form
            for (long long W = 1; W <= 4 * 64 * K + 70; ++W) {
                const int sw = 64 * K;
                const long long strips = (W + sw - 1) / sw;
                for (int vec = 0; vec < 2; ++vec) {
                    for (long long s = 0; s < strips; ++s) {
                        const StripPath path = strip_path(s, K, W, vec != 0, has_pk);
                        if (path == PATH_PK || path == PATH_FULL_PACKED || path == PATH_FULL_ELEM) {
                            // the right neighbour of lane 63 must exist unless the strip ends at the border
                            inside(right_edge_column(s, sw, W), W, "right edge", s, 63, K, W);
                        }
                        if (path != PATH_PK) {
                            inside(right_edge_column(s, sw, W), W, "right edge (clamped)", s, 63, K, W);
                            inside(left_edge_column(s, sw), W, "left edge", s, 0, K, W);
                        }
                        for (int lane = 0; lane < 64; ++lane) {
                            const long long c = s * sw + (long long)lane * K;
                            switch (path) {
                                case PATH_PK:
                                case PATH_FULL_PACKED:
                                    for (int k = 0; k < K; ++k) inside(packed_column(c, K, W, true) + k, W, "full packed", s, lane, K, W);
                                    break;
                                case PATH_LAST_PACKED:
                                    for (int k = 0; k < K; ++k) inside(packed_column(c, K, W, false) + k, W, "last packed", s, lane, K, W);
                                    break;
                                case PATH_FULL_ELEM:
                                    for (int k = 0; k < K; ++k) inside(element_column(c, k, W, true), W, "full element", s, lane, K, W);
                                    break;
                                case PATH_LAST_ELEM:
                                    for (int k = 0; k < K; ++k) inside(element_column(c, k, W, false), W, "last element", s, lane, K, W);
                                    break;
                            }
                        }
                    }
                }
            }
        }
    }
    if (failures) {
        std::fprintf(stderr, "%ld of %ld column reads outside the row\n", failures, checked);
        return 1;
    }
    std::printf("columns: ok (%ld reads)\n", checked);
    return 0;
}
