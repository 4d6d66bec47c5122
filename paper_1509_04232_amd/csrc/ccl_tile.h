// Tile-local connected components (the first step of the connectivity
// clean-up of Section 2), shared by the connectivity pass and by the
// association launch that can end in it.  Components are 4-connected pixels
// of equal label, named by their smallest raster index.
#pragma once

#include <hip/hip_runtime.h>

namespace slic {
namespace tile_ccl {

// Tiles of 32 x 32 pixels, worked by 256 threads: pixel li = threadIdx.x +
// 256 j (j < 4) of the tile, at tile row li / 32 and column li % 32, so a
// wavefront holds two whole tile rows.
constexpr int kTile = 32;
constexpr int kTilePx = kTile * kTile;
constexpr int kBlock = 256;
constexpr int kPxPerThread = kTilePx / kBlock;

template <class T>
using gptr = __attribute__((address_space(1))) T;

__device__ __forceinline__ int lds_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Merge the LDS trees of a and b, the larger root linked under the smaller
// (both walks advanced together, so that their loads overlap); a
// concurrent re-link of the root is followed through atomicMin's result.
__device__ __forceinline__ void lds_unite(int* P, int a, int b) {
    for (;;) {
        int pa = lds_load(P + a), pb = lds_load(P + b);
        while (pa != a || pb != b) {
            a = pa;
            b = pb;
            pa = lds_load(P + a);
            pb = lds_load(P + b);
        }
        if (a == b) return;
        const int lo = min(a, b), hi = max(a, b);
        const int old = atomicMin(P + hi, lo);
        if (old == hi) return;
        a = lo;
        b = old;
    }
}

// The components of the tile at (x0, y0) of a w x h image.  On entry lab[]
// holds the tile's labels in tile raster order (-1 for pixels outside the
// image), cnt[] is zero, and both are visible to the workgroup (after a
// barrier).  Local indices follow raster order inside the tile, so a local
// root (the smallest local index) is also the smallest global index of the
// component's part in the tile.  Writes P[i] = global index of i's local
// root and lroot[i] = its local index for every pixel in the image; a local
// root's size entry receives the pixel count of its part of the tile.
//
// Thread t owns column t % 32 of rows 2q + 1, 2q + 17, 2q and 2q + 16
// (q = t / 32), so each half wavefront holds one whole row at a time and
// every odd row lies below a row of the same thread.  Each pixel finds the
// head (first pixel) of its horizontal run of equal labels from a ballot of
// run starts, and a run head notes its run's length.  Union-find then
// links run heads, once per vertical overlap of two runs (at the overlap's
// first column, also from ballots), in two rounds: across the odd row
// boundaries, where both heads are the thread's own, then across the even
// ones.  Roots link under roots, and every walk starts from a run head, so
// the walks are short.
__device__ __forceinline__ void tile_components(int* lab, int* par, int* cnt, int x0, int y0,
                                                int w, int h, gptr<int>* P, gptr<int>* lroot,
                                                gptr<int>* size) {
    const int col = threadIdx.x % kTile;
    const int q = threadIdx.x / kTile;
    const int half = (threadIdx.x & 63) >= 32 ? 32 : 0;  // which row of the wavefront
    const unsigned upto = col == 31 ? 0xFFFFFFFFu : (2u << col) - 1u;
    const int rows[kPxPerThread] = {2 * q + 1, 2 * q + 17, 2 * q, 2 * q + 16};
    int head[kPxPerThread], runlen[kPxPerThread];
    unsigned unite_here = 0;  // bit j: pixel j starts a vertical overlap with the row above
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = rows[j] * kTile + col;
        // unconditional loads (clamped indices), so the three overlap
        const int v = lab[li];
        const int vl = lab[col > 0 ? li - 1 : li];
        const int vu = lab[rows[j] > 0 ? li - kTile : li];
        const bool start = col == 0 || v != vl;
        const bool inside = x0 + col < w && y0 + rows[j] < h;
        const bool above = inside && rows[j] > 0 && vu == v;
        const unsigned row_starts = static_cast<unsigned>(__ballot(start) >> half);
        const unsigned eq = static_cast<unsigned>(__ballot(above) >> half);
        head[j] = li - col + (31 - __clz(row_starts & upto));
        par[li] = head[j];
        const unsigned later = row_starts & ~upto;  // starts right of this column
        runlen[j] = start ? (later ? __ffs(later) - 1 : kTile) - col : 0;
        // the first column of each overlap: equal above, and a run start
        // or the column left of it not equal above
        if ((eq & (row_starts | ~(eq << 1))) & (1u << col)) unite_here |= 1u << j;
    }
    __syncthreads();
    // the heads of the pixels above the even rows (a head's entry may be
    // re-linked in the first round, but any node of its tree will do)
    int up[2];
#pragma unroll
    for (int j = 2; j < kPxPerThread; ++j)
        up[j - 2] = lds_load(par + (rows[j] > 0 ? rows[j] - 1 : 0) * kTile + col);
    // odd boundaries: the pixel above is the thread's own
    if (unite_here & 1u) lds_unite(par, head[0], head[2]);
    if (unite_here & 2u) lds_unite(par, head[1], head[3]);
    __syncthreads();
    // even boundaries
    if (unite_here & 4u) lds_unite(par, head[2], up[0]);
    if (unite_here & 8u) lds_unite(par, head[3], up[1]);
    __syncthreads();
    // every pixel's root, from its run head; the thread's walks advance
    // together
    int rr[kPxPerThread];
    unsigned walk = 0;
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {
        rr[j] = head[j];
        if (x0 + col < w && y0 + rows[j] < h) walk |= 1u << j;
    }
    const unsigned inside = walk;
    while (walk) {  // two levels per step, each walk halving its path for the others
        int p[kPxPerThread], gp[kPxPerThread];
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) p[j] = lds_load(par + rr[j]);
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) gp[j] = lds_load(par + p[j]);
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) {
            if (gp[j] == p[j]) walk &= ~(1u << j);
            else if (walk & (1u << j)) __hip_atomic_store(par + rr[j], gp[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            rr[j] = gp[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {
        if (!(inside & (1u << j))) {
            rr[j] = -1;
            continue;
        }
        const int r = rr[j];
        const size_t gi = static_cast<size_t>(y0 + rows[j]) * w + x0 + col;
        P[gi] = (y0 + r / kTile) * w + x0 + r % kTile;
        lroot[gi] = r;
        if (runlen[j] > 0) atomicAdd(cnt + r, runlen[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = rows[j] * kTile + col;
        if (rr[j] != li) continue;  // local roots only (pixels inside the image)
        size[static_cast<size_t>(y0 + rows[j]) * w + x0 + col] = cnt[li];
    }
}

}  // namespace tile_ccl
}  // namespace slic
