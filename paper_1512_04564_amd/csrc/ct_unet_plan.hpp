// Host-side launch plan of the warm-start U-Net's training kernels: layer shapes, the level of each
// layer, the pixel splits of the gradient reductions and the size of the partial-sum buffer they share.
// Plain C++ (no device code), so that a CPU test can run it over many batch shapes.
#pragma once

#include <algorithm>
#include <cstddef>

namespace ct {
namespace unet_plan {

constexpr int kLayers = 15;
// (c_in, c_out, kernel) in canonical order
constexpr int kShape[kLayers][3] = {{1, 32, 3},    {32, 32, 3},   {32, 64, 3},   {64, 64, 3},   {64, 128, 3},
                                    {128, 128, 3}, {128, 256, 3}, {256, 256, 3}, {384, 128, 3}, {128, 128, 3},
                                    {192, 64, 3},  {64, 64, 3},   {96, 32, 3},   {32, 32, 3},   {32, 1, 1}};
// resolution level of each layer (0: full, k: 2^-k in each direction)
constexpr int kLevel[kLayers] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0};
// pixels per split of the output- and input-layer gradient partials
constexpr int kOutPps = 4096, kInPps = 2048;

// Pixels per bias-gradient split for c channels (c / 8 dividing 256): 32 loads per thread.
constexpr int bias_pps(int c) { return 32 * (2048 / c); }

// Splits of the single-wave weight-gradient launch: about 8192 workgroups (32 per CU: its chunk loop
// waits on its loads and barriers, so occupancy hides it), at least 512 pixels per split.
inline int splits_for(size_t npix, size_t tiles)
{
    const size_t sp = std::max<size_t>(1, std::min<size_t>(npix / 512, (8192 + tiles - 1) / tiles));
    return (int)std::min<size_t>(sp, 1024);
}

// Split geometry of the single-wave weight-gradient launch: pixels per split (multiple of 64) and split count.
inline void wgrad_splits(size_t npix, int cin, int cout, int *pps, int *nsp)
{
    const size_t tiles = (size_t)9 * (cout / 32) * (cin / 32);
    const int ns = splits_for(npix, tiles);
    *pps = (int)(((npix + ns - 1) / ns + 63) / 64 * 64);
    *nsp = (int)((npix + *pps - 1) / *pps);
}

// Split cap of the nine-tap weight-gradient launch (width a multiple of 64): about 1024 workgroups of 4
// waves over the layer's channel blocks, at most one 64-pixel segment each; 0 below 64 pixels (a bound
// for a deep level of a small batch). Non-decreasing in the pixel count.
inline size_t wgrad9_split_cap(size_t npix, int cin, int cout)
{
    const size_t nseg = npix / 64, cblocks = (size_t)(cout / 32) * (cin / 32);
    return std::min<size_t>(nseg, (1024 + cblocks - 1) / cblocks);
}

// Split geometry of the nine-tap launch: 64-pixel segments per split and split count (at most the cap;
// the count itself is not monotone in the pixel count, the cap is).
inline void wgrad9_splits(size_t npix, int cin, int cout, int *cps, int *nsp)
{
    const size_t nseg = npix / 64, ns = wgrad9_split_cap(npix, cin, cout);
    if (ns == 0) {
        *cps = 1;
        *nsp = 0;
        return;
    }
    *cps = (int)((nseg + ns - 1) / ns);
    *nsp = (int)((nseg + *cps - 1) / *cps);
}

// Largest partial-sum request (floats) of any backward launch for batches up to max_n x max_h x max_w.
// Each request is at most a bound that grows with the pixel count (the split count or its cap), and the
// pixel count at level k is at most the maximum batch's count / 4^k, so the maximum batch bounds all
// smaller ones.
inline size_t part_need(int max_n, int max_h, int max_w)
{
    const size_t P1 = (size_t)max_n * max_h * max_w;
    size_t need = 0;
    for (int l = 1; l < kLayers - 1; ++l) {
        const size_t np = P1 >> (2 * kLevel[l]);
        const size_t w9 = (size_t)kShape[l][1] * 9 * kShape[l][0];
        need = std::max(need, (size_t)splits_for(np, (size_t)9 * (kShape[l][1] / 32) * (kShape[l][0] / 32)) * w9);
        need = std::max(need, wgrad9_split_cap(np, kShape[l][0], kShape[l][1]) * w9);
        need = std::max(need, ((np + bias_pps(kShape[l][1]) - 1) / bias_pps(kShape[l][1])) * (size_t)kShape[l][1]);
    }
    need = std::max(need, ((P1 + kOutPps - 1) / kOutPps) * 33);
    need = std::max(need, ((P1 + kInPps - 1) / kInPps) * 320);
    return need;
}

}  // namespace unet_plan
}  // namespace ct
