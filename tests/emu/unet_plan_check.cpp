// Sweep of the U-Net training launch plan (csrc/ct_unet_plan.hpp) over batch shapes: every backward
// launch's partial-sum request fits the buffer sized for the maximum batch, and every split geometry
// covers its pixels with no empty split. Prints the number of checks, or the first failure (exit 1).
#include <cstdio>
#include <vector>

#include "ct_unet_plan.hpp"

using namespace ct::unet_plan;

static int fails = 0;
static long checks = 0;
#define CHECK(cond, ...)                       \
    do {                                       \
        ++checks;                              \
        if (!(cond) && fails++ == 0) {         \
            std::printf("FAIL: " __VA_ARGS__); \
            std::printf("\n");                 \
        }                                      \
    } while (0)

int main()
{
    const int maxes[][3] = {{1, 8, 8},   {2, 24, 40},   {2, 64, 64},   {3, 96, 128},  {1, 512, 512},
                            {4, 512, 512}, {2, 256, 256}, {1, 1024, 64}, {5, 40, 640}, {8, 512, 512}};
    for (const auto &m : maxes) {
        const size_t need = part_need(m[0], m[1], m[2]);
        for (int n = 1; n <= m[0]; ++n)
            for (int h = 8; h <= m[1]; h += (m[1] > 64 ? 56 : 8))
                for (int w = 8; w <= m[2]; w += (m[2] > 64 ? 56 : 8)) {
                    const size_t P1 = (size_t)n * h * w;
                    for (int l = 1; l < kLayers - 1; ++l) {
                        const int lv = kLevel[l], hl = h >> lv, wl = w >> lv;
                        const size_t np = (size_t)n * hl * wl;
                        const int cin = kShape[l][0], cout = kShape[l][1];
                        const size_t w9 = (size_t)cout * 9 * cin;
                        if (wl % 64 == 0) {
                            int cps, nsp;
                            wgrad9_splits(np, cin, cout, &cps, &nsp);
                            const size_t nseg = np / 64;
                            CHECK(nsp >= 1 && cps >= 1, "nine-tap split of %zu px: %d x %d", np, nsp, cps);
                            CHECK((size_t)nsp * cps >= nseg && (size_t)(nsp - 1) * cps < nseg,
                                  "nine-tap cover %zu segments with %d x %d", nseg, nsp, cps);
                            CHECK((size_t)nsp * w9 <= need, "nine-tap request %zu > %zu (%d %d %d, layer %d)",
                                  (size_t)nsp * w9, need, n, h, w, l);
                        } else {
                            int pps, nsp;
                            wgrad_splits(np, cin, cout, &pps, &nsp);
                            CHECK(pps % 64 == 0 && nsp >= 1, "split of %zu px: %d x %d", np, nsp, pps);
                            CHECK((size_t)nsp * pps >= np && (size_t)(nsp - 1) * pps < np, "cover %zu px with %d x %d",
                                  np, nsp, pps);
                            CHECK((size_t)nsp * w9 <= need, "request %zu > %zu (%d %d %d, layer %d)",
                                  (size_t)nsp * w9, need, n, h, w, l);
                        }
                        const size_t nb = (np + bias_pps(cout) - 1) / bias_pps(cout);
                        CHECK(nb * cout <= need, "bias request %zu > %zu", nb * cout, need);
                    }
                    CHECK(((P1 + kOutPps - 1) / kOutPps) * 33 <= need, "output-layer request");
                    CHECK(((P1 + kInPps - 1) / kInPps) * 320 <= need, "input-layer request");
                }
    }
    std::printf("%ld checks, %d failed\n", checks, fails);
    return fails ? 1 : 0;
}
