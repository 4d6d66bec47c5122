// Connectivity clean-up (Section 2, final step), under a canonical rule that
// a sequential implementation reproduces exactly:
//  1. 4-connected components of equal label, each named by its smallest
//     raster index (its root pixel);
//  2. component sizes;
//  3. a component below the size threshold, other than the one holding
//     pixel 0, joins the component of the pixel left of its root (above it
//     when the root starts a row); joins point to earlier roots, so they form
//     a forest;
//  4. each component takes its tree root's segment, and segments are
//     numbered 0.. in raster order of their roots.
//
// GPU structure: concurrent union-find whose links always point from a
// larger to a smaller index (so a tree's root is its minimum), first inside
// 32 x 32 tiles in LDS, then across tile borders in global memory; the joins
// of step 3 recorded per small root as links in the rank array and followed
// (with path splitting) by the relabel pass; ballot counts and prefix sums
// over the surviving roots for the numbering.  All integer, so the result
// is exact.
#include "ccl_tile.h"
#include "slic_internal.h"

namespace slic {
namespace {

constexpr int kBlock = 256;

// Global (device) memory as a named address space.  Descriptors read from
// a batch table hold generic pointers; accesses through them would compile
// to flat instructions, which also count against the LDS wait counter, so
// every kernel takes its arrays as global-address-space pointers.
template <class T>
using gmem = __attribute__((address_space(1))) T;

template <class T>
__device__ __forceinline__ gmem<T>* as_global(T* p) {
    return (gmem<T>*)p;
}

__device__ __forceinline__ int load_relaxed(gmem<int>* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int atomic_min(gmem<int>* p, int v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The roots of a and b, the two walks advanced together so that their
// loads overlap.
__device__ __forceinline__ void find_roots(gmem<int>* P, int& a, int& b) {
    int pa = load_relaxed(P + a), pb = load_relaxed(P + b);
    while (pa != a || pb != b) {
        a = pa;
        b = pb;
        pa = load_relaxed(P + a);
        pb = load_relaxed(P + b);
    }
}

// Merge the trees of a and b, linking the larger root under the smaller.
// If another thread re-linked the root meanwhile, atomicMin returns that new
// parent and the merge continues from it.
__device__ void unite(gmem<int>* P, int a, int b) {
    bool done;
    do {
        find_roots(P, a, b);
        if (a < b) {
            const int old = atomic_min(P + b, a);
            done = old == b;
            b = old;
        } else if (b < a) {
            const int old = atomic_min(P + a, b);
            done = old == a;
            a = old;
        } else {
            done = true;
        }
    } while (!done);
}

// ---- components in three steps: union-find inside 32 x 32 tiles in LDS,
// unions across tile borders in global memory, then every pixel resolves its
// root and the tile adds its pixel counts per root.
constexpr int kTile = tile_ccl::kTile;
constexpr int kTilePx = tile_ccl::kTilePx;
constexpr int kPxPerThread = tile_ccl::kPxPerThread;
static_assert(kBlock == tile_ccl::kBlock, "the tile passes use the shared tile shape");

// The image of tile number idx of a launch and the tile's (x, y) among the
// image's 32 x 32 tiles: from the kernel argument (one image) or, for a
// batch, from the image table through the tile-to-image map.
__device__ __forceinline__ void resolve_tile(const CclImage& single, const CclMap& map, int idx,
                                             CclImage* g, int* bx, int* by) {
    int local = idx;
    if (map.images) {
        const int img = map.tile_image[idx];
        *g = map.images[img];
        local -= map.tile_first[img];
    } else {
        *g = single;
    }
    *bx = local % g->tiles_x;
    *by = local / g->tiles_x;
}

// The tile passes: one image on a two-dimensional grid of tiles (kBatch
// false: no table lookups and no division on the way in), or a batch on a
// one-dimensional grid through the map.
template <bool kBatch>
__device__ __forceinline__ void tile_of_launch(const CclImage& single, const CclMap& map,
                                               CclImage* g, int* bx, int* by) {
    if constexpr (kBatch) {
        resolve_tile(single, map, blockIdx.x, g, bx, by);
    } else {
        *g = single;
        *bx = blockIdx.x;
        *by = blockIdx.y;
    }
}

// Likewise for the passes over runs of kMergeBlock consecutive pixels.
template <bool kBatch>
__device__ __forceinline__ void resolve_block(const CclImage& single, const CclMap& map,
                                              CclImage* g, int* blk) {
    if constexpr (kBatch) {
        const int img = map.blk_image[blockIdx.x];
        *g = map.images[img];
        *blk = static_cast<int>(blockIdx.x) - map.blk_first[img];
    } else {
        *g = single;
        *blk = blockIdx.x;
    }
}

// Tile-local components of the association labels: the tile's labels into
// LDS, then tile_ccl::tile_components (P, lroot and the local roots' sizes).
// The association launch that ends a segmentation can do this itself for
// 32 x 32 tiles; the pass is then skipped.
template <bool kBatch>
__global__ __launch_bounds__(kBlock) void ccl_local_kernel(CclImage single, CclMap map) {
    __shared__ int lab[kTilePx];
    __shared__ int par[kTilePx];
    __shared__ int cnt[kTilePx];
    CclImage g;
    int bx, by;
    tile_of_launch<kBatch>(single, map, &g, &bx, &by);
    gmem<const int32_t>* __restrict__ labels = as_global(g.labels);
    gmem<int>* __restrict__ P = as_global(g.comp);
    gmem<int>* __restrict__ lroot = as_global(g.lroot);
    gmem<int>* __restrict__ size = as_global(g.size);
    const int w = g.w, h = g.h;
    const int x0 = bx * kTile, y0 = by * kTile;
    const int col = threadIdx.x % kTile;
    int v[kPxPerThread];
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {  // clamped: the loads are issued together
        const int li = threadIdx.x + j * kBlock;
        const int x = x0 + col, y = y0 + li / kTile;
        v[j] = labels[static_cast<size_t>(min(y, h - 1)) * w + min(x, w - 1)];
    }
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = threadIdx.x + j * kBlock;
        const int x = x0 + col, y = y0 + li / kTile;
        lab[li] = (x < w && y < h) ? v[j] : -1;
        cnt[li] = 0;
    }
    __syncthreads();
    tile_ccl::tile_components(lab, par, cnt, x0, y0, w, h, P, lroot, size);
}

// Unions across the left and top borders of every tile.
template <bool kBatch>
__global__ __launch_bounds__(2 * kTile) void ccl_border_kernel(CclImage single, CclMap map) {
    CclImage g;
    int bx, by;
    tile_of_launch<kBatch>(single, map, &g, &bx, &by);
    gmem<const int32_t>* __restrict__ labels = as_global(g.labels);
    gmem<int>* P = as_global(g.comp);
    const int w = g.w, h = g.h;
    const int x0 = bx * kTile, y0 = by * kTile;
    const int t = threadIdx.x;
    if (t < kTile) {
        const int x = x0, y = y0 + t;
        if (x0 == 0 || y >= h) return;
        const int i = y * w + x;
        if (labels[i] == labels[i - 1]) unite(P, i, i - 1);
    } else {
        const int x = x0 + t - kTile, y = y0;
        if (y0 == 0 || x >= w) return;
        const int i = y * w + x;
        if (labels[i] == labels[i - w]) unite(P, i, i - w);
    }
}

// comp[i] = P[i] = root of i (the component's smallest index).  Only the
// tile's local roots walk the forest (the thread's walks advanced together,
// with unconditional loads, so that they overlap); every pixel then takes
// its local root's result from LDS.  A local root that is not its
// component's root adds its part's pixel count (its size entry, from the
// tile-local pass) to the root's entry, which holds the root's own part.
template <bool kBatch>
__global__ __launch_bounds__(kBlock) void ccl_flatten_kernel(CclImage single, CclMap map) {
    __shared__ int root[kTilePx];
    CclImage g;
    int bx, by;
    tile_of_launch<kBatch>(single, map, &g, &bx, &by);
    gmem<int>* P = as_global(g.comp);
    gmem<const int>* __restrict__ lroot = as_global(g.lroot);
    gmem<int>* size = as_global(g.size);
    const int w = g.w, h = g.h;
    const int x0 = bx * kTile, y0 = by * kTile;
    int lr[kPxPerThread], x[kPxPerThread], self[kPxPerThread];
    bool in[kPxPerThread];
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = threadIdx.x + j * kBlock;
        const int px = x0 + li % kTile, py = y0 + li / kTile;
        in[j] = px < w && py < h;
        lr[j] = lroot[static_cast<size_t>(min(py, h - 1)) * w + min(px, w - 1)];
        // a local root starts a walk from its own pixel; others stand on
        // pixel 0, which is always a root
        self[j] = in[j] && lr[j] == li ? py * w + px : 0;
        x[j] = self[j];
    }
    unsigned live = 0u;
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j)
        if (x[j] != 0) live |= 1u << j;
    while (live) {
        int p[kPxPerThread];
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) p[j] = load_relaxed(P + x[j]);
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) {
            if (!(live & (1u << j))) continue;
            if (p[j] == x[j]) live &= ~(1u << j);
            x[j] = p[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = threadIdx.x + j * kBlock;
        if (!(in[j] && lr[j] == li)) continue;
        root[li] = x[j];
        if (x[j] != self[j])  // pixel 0 is always its own root, so self 0 never adds
            __hip_atomic_fetch_add(size + x[j], size[self[j]], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPxPerThread; ++j) {
        if (!in[j]) continue;
        const int li = threadIdx.x + j * kBlock;
        const size_t gi = static_cast<size_t>(y0 + li / kTile) * w + x0 + li % kTile;
        __hip_atomic_store(P + gi, root[lr[j]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Joins.  A small component (other than the one holding pixel 0) joins the
// component of the pixel left of its root r, or above r at a row start;
// both have smaller roots, so the joins form a forest whose tree roots are
// the smallest indices of their trees and are exactly the components that
// are not small (or hold pixel 0).  After the flatten pass every entry of
// comp holds its pixel's component root and nothing writes comp any more.
//
// The merge launch has two kinds of workgroups.  The first n_number number
// the surviving roots: each covers kMergeBlock consecutive pixels (thread t
// handles pixels t, t + kBlock, ...), gives its survivors their rank in
// raster order among the workgroup's survivors (ballot prefix counts) and
// stores their count.  The others each take a 32 x 32 tile and record the
// join of every small root in it as rank[r] = -2 - target, where target is
// the first root along the chain of joins that is not a small root of the
// same tile: the joins inside a tile are followed in LDS, so the relabel
// pass only walks the joins that cross tiles (on noisy label maps a chain of
// small components, each joining its left neighbour, can be dozens long).
// Loads are unconditional (positions past the image are clamped) so that a
// thread's loads are issued together rather than one branch at a time.
constexpr int kMergePx = 4;
constexpr int kMergeBlock = kBlock * kMergePx;

__device__ __forceinline__ bool is_small(const CclImage& g, int sz) {
    return g.min_segment > 0 ? sz < g.min_segment : 4ll * sz < g.S2;
}

template <bool kBatch>
__global__ __launch_bounds__(kBlock) void ccl_merge_kernel(CclImage single, CclMap map,
                                                           int n_number) {
    __shared__ int part[kMergePx * (kBlock / 64)];
    __shared__ int link[kTilePx];
    CclImage g;
    if (static_cast<int>(blockIdx.x) >= n_number) {
        // ---- joins of the small roots of one tile
        int bx, by;
        const int idx = static_cast<int>(blockIdx.x) - n_number;
        if constexpr (kBatch) {
            resolve_tile(single, map, idx, &g, &bx, &by);
        } else {
            g = single;
            bx = idx % g.tiles_x;
            by = idx / g.tiles_x;
        }
        const int w = g.w, h = g.h;
        const int x0 = bx * kTile, y0 = by * kTile;
        gmem<const int>* __restrict__ comp = as_global(g.comp);
        gmem<const int>* __restrict__ size = as_global(g.size);
        gmem<int>* __restrict__ rank = as_global(g.rank);
        int gi[kPxPerThread], t[kPxPerThread], sz[kPxPerThread];
        bool small[kPxPerThread], root[kPxPerThread];
        // the roots first (all loads issued together), then the size and the
        // join target, which other pixels (most are not roots) read from
        // pixel 0 instead: the loads stay unconditional, so they are issued
        // together, and non-roots fetch one shared line
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) {
            const int li = threadIdx.x + j * kBlock;
            const int px = x0 + li % kTile, py = y0 + li / kTile;
            gi[j] = min(py, h - 1) * w + min(px, w - 1);
            const int c = comp[gi[j]];
            root[j] = px < w && py < h && c == gi[j];
        }
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) {
            const int q = gi[j] % w > 0 ? gi[j] - 1 : max(gi[j] - w, 0);  // left, or above
            sz[j] = size[root[j] ? gi[j] : 0];
            t[j] = comp[root[j] ? q : 0];
        }
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) {
            const int li = threadIdx.x + j * kBlock;
            small[j] = root[j] && gi[j] != 0 && is_small(g, sz[j]);
            // link: a tile slot for a target inside the tile, -4 - target for
            // one outside, -1 for a surviving root, -2 for a pixel that is
            // not a root (never reached: targets are roots)
            int l = root[j] ? -1 : -2;
            if (small[j]) {
                const int ty = t[j] / w, tx = t[j] - ty * w;
                const bool inside = tx >= x0 && tx < x0 + kTile && ty >= y0 && ty < y0 + kTile;
                l = inside ? (ty - y0) * kTile + (tx - x0) : -4 - t[j];
            }
            link[li] = l;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPxPerThread; ++j) {
            if (!small[j]) continue;
            int l = link[threadIdx.x + j * kBlock], slot = -1;
            while (l >= 0) {  // links point to smaller slots: the walk ends
                slot = l;
                l = link[slot];
            }
            const int target = l <= -4 ? -4 - l : (y0 + slot / kTile) * w + x0 + slot % kTile;
            rank[gi[j]] = -2 - target;
        }
        return;
    }
    // ---- numbering of the surviving roots of kMergeBlock consecutive pixels
    int blk;
    resolve_block<kBatch>(single, map, &g, &blk);
    const int n = g.w * g.h;
    gmem<const int>* __restrict__ comp = as_global(g.comp);
    gmem<const int>* __restrict__ size = as_global(g.size);
    gmem<int>* __restrict__ rank = as_global(g.rank);
    const int base = blk * kMergeBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool survives[kMergePx], root[kMergePx];
#pragma unroll
    for (int j = 0; j < kMergePx; ++j) {
        const int r = base + j * kBlock;
        root[j] = r < n && comp[min(r, n - 1)] == r;
    }
#pragma unroll
    for (int j = 0; j < kMergePx; ++j) {
        const int r = base + j * kBlock;
        const int sz = size[root[j] ? r : 0];  // non-roots share one line
        survives[j] = root[j] && (r == 0 || !is_small(g, sz));
    }
    unsigned long long ballot[kMergePx];
#pragma unroll
    for (int j = 0; j < kMergePx; ++j) {
        ballot[j] = __ballot(survives[j]);
        if (lane == 0) part[j * (kBlock / 64) + wave] = __popcll(ballot[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMergePx; ++j) {
        if (!survives[j]) continue;
        int offset = 0;  // survivors in the (pass, wave) groups before this one
        for (int q = 0; q < j * (kBlock / 64) + wave; ++q) offset += part[q];
        rank[base + j * kBlock] = offset + __popcll(ballot[j] & ((1ull << lane) - 1ull));
    }
    if (threadIdx.x == 0) {
        int total = 0;
        for (int q = 0; q < kMergePx * (kBlock / 64); ++q) total += part[q];
        as_global(g.block_count)[blk] = total;
    }
}

// One workgroup: exclusive scan of the per-block counts in place; the total
// is the number of segments.
__global__ __launch_bounds__(kBlock) void ccl_scan_kernel(int nblocks, int* __restrict__ count,
                                                          int* __restrict__ n_segments) {
    __shared__ int part[kBlock];
    const int per = (nblocks + kBlock - 1) / kBlock;
    const int lo = threadIdx.x * per, hi = min(lo + per, nblocks);
    int sum = 0;
    for (int j = lo; j < hi; ++j) sum += count[j];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {  // Hillis-Steele inclusive scan
        const int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    for (int j = lo; j < hi; ++j) {
        const int c = count[j];
        count[j] = run;
        run += c;
    }
    if (threadIdx.x == kBlock - 1 && n_segments) *n_segments = part[kBlock - 1];
}

// Up to this many runs of kMergeBlock pixels every relabel workgroup scans
// the runs' survivor counts itself, in LDS, and the one-workgroup scan launch
// is skipped; beyond it the scan kernel runs first.
constexpr int kFusedScanMax = 4096;
constexpr int kFusedScanSmall = 1024;  // a variant with fewer count loads per thread

// Final labels: rank of the pixel's surviving root plus the number of
// survivors in earlier runs.  comp[i] is the pixel's component
// root; a surviving root carries its rank, a joined one -2 - (the root it
// joins), and the joins are followed to the tree root.  Same pixel-to-thread
// map as the merge pass.  With SQ > 0 (up to SQ * kBlock runs), block_count
// holds the merge pass's counts and every workgroup derives the offsets
// itself (workgroup 0 also stores the total); with SQ = 0 it holds the
// offsets already.
template <int SQ, bool kBatch>
__global__ __launch_bounds__(kBlock) void ccl_relabel_kernel(CclImage single, CclMap map) {
    extern __shared__ int s_off[];  // SQ > 0: nblocks offsets
    __shared__ int wave_part[kBlock / 64];
    CclImage g;
    int blk;
    resolve_block<kBatch>(single, map, &g, &blk);
    const int n = g.w * g.h, nblocks = g.nmerge;
    gmem<const int>* __restrict__ comp = as_global(g.comp);
    gmem<int>* rank = as_global(g.rank);
    gmem<const int>* __restrict__ block_count = as_global(g.block_count);
    gmem<int32_t>* __restrict__ out = as_global(g.out);
    const int base = blk * kMergeBlock + threadIdx.x;
    int r[kMergePx], k[kMergePx];
#pragma unroll
    for (int j = 0; j < kMergePx; ++j)  // clamped: loads issued together
        r[j] = comp[min(base + j * kBlock, n - 1)];
#pragma unroll
    for (int j = 0; j < kMergePx; ++j) k[j] = rank[r[j]];
    if constexpr (SQ > 0) {
        // exclusive prefix sums of the counts into s_off: coalesced loads
        // into LDS, each thread sums a run of consecutive counts, the runs'
        // sums are scanned with shuffles in each wavefront and then across
        // the wavefronts, and each thread writes its run's offsets back
        constexpr int kQ = SQ;
        int cnt[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q)  // clamped, so every load is issued at once
            cnt[q] = block_count[min(static_cast<int>(threadIdx.x) + q * kBlock, nblocks - 1)];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int j = threadIdx.x + q * kBlock;
            if (j < nblocks) s_off[j] = cnt[q];
        }
        __syncthreads();
        const int per = (nblocks + kBlock - 1) / kBlock;
        const int lo = min(static_cast<int>(threadIdx.x) * per, nblocks);
        const int hi = min(lo + per, nblocks);
        int sum = 0;
        for (int j = lo; j < hi; ++j) sum += s_off[j];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        int inc = sum;
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(inc, d);
            if (lane >= d) inc += v;
        }
        if (lane == 63) wave_part[wave] = inc;
        __syncthreads();
        int run = inc - sum, total = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            if (q < wave) run += wave_part[q];
            total += wave_part[q];
        }
        for (int j = lo; j < hi; ++j) {
            const int c = s_off[j];
            s_off[j] = run;
            run += c;
        }
        __syncthreads();
        if (blk == 0 && threadIdx.x == 0 && g.n_segments) *as_global(g.n_segments) = total;
    }
    // Follow the joins to a surviving root, one rank load per step, the
    // thread's walks advanced together (finished ones reload their root,
    // harmlessly) so that their loads overlap.  Each step also re-links the
    // root visited before to the current root's target (path splitting: the
    // target is an ancestor, so concurrent walks stay correct), so walks
    // that pass the same chain of joins later find it shorter.
    int prev[kMergePx];
#pragma unroll
    for (int j = 0; j < kMergePx; ++j) prev[j] = -1;
    unsigned live = 0u;
#pragma unroll
    for (int j = 0; j < kMergePx; ++j)
        if (k[j] < 0) live |= 1u << j;
    while (live) {
        int nx[kMergePx], kn[kMergePx];
#pragma unroll
        for (int j = 0; j < kMergePx; ++j) nx[j] = k[j] < 0 ? -2 - k[j] : r[j];
#pragma unroll
        for (int j = 0; j < kMergePx; ++j) kn[j] = rank[nx[j]];
#pragma unroll
        for (int j = 0; j < kMergePx; ++j) {
            if (!(live & (1u << j))) continue;
            if (prev[j] >= 0) rank[prev[j]] = k[j];
            prev[j] = r[j];
            r[j] = nx[j];
            k[j] = kn[j];
            if (k[j] >= 0) live &= ~(1u << j);
        }
    }
    auto offset_of = [&](int root) {
        if constexpr (SQ > 0) {
            return s_off[root / kMergeBlock];
        } else {
            return block_count[root / kMergeBlock];
        }
    };
#pragma unroll
    for (int j = 0; j < kMergePx; ++j) {
        const int i = base + j * kBlock;
        if (i < n) out[i] = k[j] + offset_of(r[j]);
    }
}

}  // namespace

int scan_tiles_for(int n) { return (n + kMergeBlock - 1) / kMergeBlock; }

CclImage ccl_image(const Workspace& ws, int32_t w, int32_t h, const Grid& g, int32_t min_segment,
                   int32_t* labels_out, int32_t* n_segments) {
    CclImage c;
    c.labels = ws.labels;
    c.out = labels_out;
    c.comp = ws.ccl0;   // local roots, then component roots
    c.size = ws.ccl1;   // component sizes
    c.rank = ws.ccl2;   // ranks of the surviving roots, join links of the others
    c.lroot = ws.ccl3;  // local roots (index inside the tile)
    c.block_count = ws.scan;  // per-block surviving roots (then their offsets)
    c.n_segments = n_segments;
    c.w = w;
    c.h = h;
    c.S2 = static_cast<long long>(g.S) * g.S;
    c.min_segment = min_segment;
    c.tiles_x = (w + kTile - 1) / kTile;
    c.nmerge = scan_tiles_for(w * h);
    return c;
}

int ccl_tiles_for(int32_t w, int32_t h) {
    return ((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile);
}

bool ccl_batch_supported(int32_t w, int32_t h) { return scan_tiles_for(w * h) <= kFusedScanMax; }

#define SLIC_STEP(name, ...)                                 \
    do {                                                     \
        KernelTimer t_(name, s);                             \
        __VA_ARGS__;                                         \
        if ((e = hipGetLastError()) != hipSuccess) return e; \
    } while (0)

hipError_t launch_connectivity(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                               int32_t min_segment, int32_t* labels_out, int32_t* n_segments,
                               hipStream_t s, bool local_done) {
    const CclImage c = ccl_image(ws, w, h, g, min_segment, labels_out, n_segments);
    const CclMap none{};
    hipError_t e;
    const int tiles = ccl_tiles_for(w, h);
    const dim3 grid((w + kTile - 1) / kTile, (h + kTile - 1) / kTile);
    if (!local_done)
        SLIC_STEP("ccl_local", ccl_local_kernel<false><<<grid, kBlock, 0, s>>>(c, none));
    SLIC_STEP("ccl_border", ccl_border_kernel<false><<<grid, 2 * kTile, 0, s>>>(c, none));
    SLIC_STEP("ccl_flatten", ccl_flatten_kernel<false><<<grid, kBlock, 0, s>>>(c, none));
    SLIC_STEP("ccl_merge",
              ccl_merge_kernel<false><<<c.nmerge + tiles, kBlock, 0, s>>>(c, none, c.nmerge));
    const size_t lds = c.nmerge * sizeof(int);
    if (c.nmerge <= kFusedScanSmall) {
        SLIC_STEP("ccl_relabel",
                  ccl_relabel_kernel<kFusedScanSmall / kBlock, false><<<c.nmerge, kBlock, lds, s>>>(
                      c, none));
    } else if (c.nmerge <= kFusedScanMax) {
        SLIC_STEP("ccl_relabel",
                  ccl_relabel_kernel<kFusedScanMax / kBlock, false><<<c.nmerge, kBlock, lds, s>>>(
                      c, none));
    } else {
        SLIC_STEP("ccl_scan", ccl_scan_kernel<<<1, kBlock, 0, s>>>(c.nmerge, c.block_count,
                                                                   c.n_segments));
        SLIC_STEP("ccl_relabel", ccl_relabel_kernel<0, false><<<c.nmerge, kBlock, 0, s>>>(c, none));
    }
    return hipSuccess;
}

hipError_t launch_connectivity_batch(const CclMap& map, int total_tiles, int total_blocks,
                                     int max_nmerge, hipStream_t s) {
    if (!map.images || max_nmerge > kFusedScanMax) return hipErrorInvalidValue;
    const CclImage unused{};
    hipError_t e;
    SLIC_STEP("ccl_local", ccl_local_kernel<true><<<total_tiles, kBlock, 0, s>>>(unused, map));
    SLIC_STEP("ccl_border",
              ccl_border_kernel<true><<<total_tiles, 2 * kTile, 0, s>>>(unused, map));
    SLIC_STEP("ccl_flatten",
              ccl_flatten_kernel<true><<<total_tiles, kBlock, 0, s>>>(unused, map));
    SLIC_STEP("ccl_merge", ccl_merge_kernel<true><<<total_blocks + total_tiles, kBlock, 0, s>>>(
                               unused, map, total_blocks));
    const size_t lds = max_nmerge * sizeof(int);
    if (max_nmerge <= kFusedScanSmall) {
        SLIC_STEP("ccl_relabel",
                  ccl_relabel_kernel<kFusedScanSmall / kBlock, true><<<total_blocks, kBlock, lds, s>>>(
                      unused, map));
    } else {
        SLIC_STEP("ccl_relabel",
                  ccl_relabel_kernel<kFusedScanMax / kBlock, true><<<total_blocks, kBlock, lds, s>>>(
                      unused, map));
    }
    return hipSuccess;
}

#undef SLIC_STEP

// Stray-pixel filter (Section 3's clean-up: two one-thread-per-pixel passes
// of one kernel).  A pixel none of whose 4-neighbours inside the image shares
// its label takes the label that occurs most often among them, ties going to
// the first in the order up, left, right, down.  Each pass reads one map and
// writes the other.
namespace {

__global__ __launch_bounds__(kBlock) void stray_kernel(const int32_t* __restrict__ in, int w, int h,
                                                       int32_t* __restrict__ out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= w * h) return;
    const int x = i % w, y = i / w;
    const int32_t own = in[i];
    int32_t nb[4];
    int n = 0;
    if (y > 0) nb[n++] = in[i - w];
    if (x > 0) nb[n++] = in[i - 1];
    if (x + 1 < w) nb[n++] = in[i + 1];
    if (y + 1 < h) nb[n++] = in[i + w];
    bool stray = n > 0;
    for (int j = 0; j < n; ++j) stray = stray && nb[j] != own;
    int32_t v = own;
    if (stray) {
        int best_count = 0;
        for (int j = 0; j < n; ++j) {
            int count = 0;
            for (int k = 0; k < n; ++k) count += nb[k] == nb[j];
            if (count > best_count) {
                best_count = count;
                v = nb[j];
            }
        }
    }
    out[i] = v;
}

__global__ __launch_bounds__(kBlock) void copy_labels_kernel(const int32_t* __restrict__ in, int n,
                                                             int32_t* __restrict__ out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = in[i];
}

}  // namespace

hipError_t launch_stray_filter(const Workspace& ws, int32_t w, int32_t h, int32_t* labels,
                               int32_t passes, hipStream_t s) {
    const int n = w * h;
    const int nb = (n + kBlock - 1) / kBlock;
    int32_t* buf[2] = {labels, ws.ccl0};
    for (int p = 0; p < passes; ++p) {
        KernelTimer t("stray", s);
        stray_kernel<<<nb, kBlock, 0, s>>>(buf[p & 1], w, h, buf[(p + 1) & 1]);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (passes & 1) {
        KernelTimer t("stray_copy", s);
        copy_labels_kernel<<<nb, kBlock, 0, s>>>(ws.ccl0, n, labels);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace slic
