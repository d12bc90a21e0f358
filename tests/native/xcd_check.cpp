// xcd_check.cpp -- host check that the dataflow kernel's XCD-aware workgroup
// numbering (xcd_block in the library's internal header) is a bijection of
// the grid onto itself for every grid size, first workgroup of the
// one-lane-per-node range and line group size the launches can use, and
// that it gives each XCD whole spans of g consecutive slots.  Test
// infrastructure, built and run by the CPU test suite.
#include <cstdio>
#include <vector>

#include "internal.h"

int main() {
    using siminf::xcd_block;
    using siminf::XCDS;
    long checked = 0;
    for (int g : {0, 1, 2, 4, 8}) {
        for (int nblk = 1; nblk <= 2500; nblk += (nblk < 300 ? 1 : 37)) {
            for (int b0 = 0; b0 <= nblk && b0 <= 70; b0 += (b0 < 20 ? 1 : 7)) {
                std::vector<int> seen(nblk, 0);
                for (int b = 0; b < nblk; ++b) {
                    const int x = xcd_block(b, b0, nblk, g);
                    if (x < 0 || x >= nblk || seen[x]++) {
                        std::printf("not a bijection: g %d nblk %d b0 %d b %d -> %d\n", g, nblk, b0, b, x);
                        return 1;
                    }
                    // workgroup b runs on XCD b % 8; inside whole spans, the g
                    // slots an XCD receives in one span are consecutive
                    const int a = (b0 + XCDS - 1) / XCDS * XCDS;
                    if (g > 1 && b >= a) {
                        const int span = XCDS * g;
                        const int full_end = a + (nblk - a) / span * span;
                        if (b < full_end) {
                            const int r = b - a, rem = r % span;
                            const int first = a + (r - rem) + (rem % XCDS) * g;
                            if (x < first || x >= first + g || (x - first) != rem / XCDS) {
                                std::printf("span layout: g %d nblk %d b0 %d b %d -> %d\n", g, nblk, b0, b, x);
                                return 1;
                            }
                        } else if (x != b) {
                            std::printf("tail moved: g %d nblk %d b0 %d b %d -> %d\n", g, nblk, b0, b, x);
                            return 1;
                        }
                    } else if (x != b) {
                        std::printf("moved outside the range: g %d nblk %d b0 %d b %d -> %d\n", g, nblk, b0, b, x);
                        return 1;
                    }
                    ++checked;
                }
            }
        }
    }
    std::printf("ok %ld\n", checked);
    return 0;
}
