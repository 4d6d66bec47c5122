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
// 32 x 32 tiles in LDS, then across tile borders in global memory; path
// following for the joins; an exclusive prefix sum over the surviving roots
// for the numbering.  All integer, so the result is exact.
#include "slic_internal.h"

namespace slic {
namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int load_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int find_root(int* P, int x) {
    int p = load_relaxed(P + x);
    while (p != x) {
        x = p;
        p = load_relaxed(P + x);
    }
    return x;
}

// Merge the trees of a and b, linking the larger root under the smaller.
// If another thread re-linked the root meanwhile, atomicMin returns that new
// parent and the merge continues from it.
__device__ void unite(int* P, int a, int b) {
    bool done;
    do {
        a = find_root(P, a);
        b = find_root(P, b);
        if (a < b) {
            const int old = atomicMin(P + b, a);
            done = old == b;
            b = old;
        } else if (b < a) {
            const int old = atomicMin(P + a, b);
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
constexpr int kTile = 32;
constexpr int kTilePx = kTile * kTile;
constexpr int kPxPerThread = kTilePx / kBlock;

__device__ __forceinline__ int lds_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int lds_find(int* P, int x) {
    int p = lds_load(P + x);
    while (p != x) {
        x = p;
        p = lds_load(P + x);
    }
    return x;
}

__device__ void lds_unite(int* P, int a, int b) {
    bool done;
    do {
        a = lds_find(P, a);
        b = lds_find(P, b);
        if (a < b) {
            const int old = atomicMin(P + b, a);
            done = old == b;
            b = old;
        } else if (b < a) {
            const int old = atomicMin(P + a, b);
            done = old == a;
            a = old;
        } else {
            done = true;
        }
    } while (!done);
}

// Tile-local components.  Local indices follow raster order inside the
// tile, so a local root (the smallest local index) is also the smallest
// global index of the component's part in the tile.  Writes P[i] = global
// index of i's local root, lroot[i] = its local index, and clears size[i].
__global__ __launch_bounds__(kBlock) void ccl_local_kernel(const int32_t* __restrict__ labels,
                                                           int w, int h, int* __restrict__ P,
                                                           int* __restrict__ lroot,
                                                           int* __restrict__ size) {
    __shared__ int lab[kTilePx];
    __shared__ int par[kTilePx];
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = threadIdx.x + j * kBlock;
        const int x = x0 + li % kTile, y = y0 + li / kTile;
        lab[li] = (x < w && y < h) ? labels[static_cast<size_t>(y) * w + x] : -1;
        par[li] = li;
    }
    __syncthreads();
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = threadIdx.x + j * kBlock;
        const int x = x0 + li % kTile, y = y0 + li / kTile;
        if (x >= w || y >= h) continue;
        const int v = lab[li];
        if (li % kTile > 0 && lab[li - 1] == v) lds_unite(par, li, li - 1);
        if (li >= kTile && lab[li - kTile] == v) lds_unite(par, li, li - kTile);
    }
    __syncthreads();
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = threadIdx.x + j * kBlock;
        const int x = x0 + li % kTile, y = y0 + li / kTile;
        if (x >= w || y >= h) continue;
        const int r = lds_find(par, li);
        const size_t gi = static_cast<size_t>(y) * w + x;
        P[gi] = (y0 + r / kTile) * w + x0 + r % kTile;
        lroot[gi] = r;
        size[gi] = 0;
    }
}

// Unions across the left and top borders of every tile.
__global__ __launch_bounds__(2 * kTile) void ccl_border_kernel(const int32_t* __restrict__ labels,
                                                               int w, int h, int* P) {
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
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

// comp[i] = P[i] = root of i (the component's smallest index); the tile adds
// its pixel count per local root to size[root].
__global__ __launch_bounds__(kBlock) void ccl_flatten_kernel(int w, int h, int* P,
                                                             const int* __restrict__ lroot,
                                                             int* __restrict__ size) {
    __shared__ int cnt[kTilePx];
    __shared__ int root[kTilePx];
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
    for (int j = 0; j < kPxPerThread; ++j) cnt[threadIdx.x + j * kBlock] = 0;
    __syncthreads();
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = threadIdx.x + j * kBlock;
        const int x = x0 + li % kTile, y = y0 + li / kTile;
        if (x >= w || y >= h) continue;
        const size_t gi = static_cast<size_t>(y) * w + x;
        const int lr = lroot[gi];
        const int r = find_root(P, (y0 + lr / kTile) * w + x0 + lr % kTile);
        atomicAdd(cnt + lr, 1);
        root[lr] = r;
        __hip_atomic_store(P + gi, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    for (int j = 0; j < kPxPerThread; ++j) {
        const int li = threadIdx.x + j * kBlock;
        const int c = cnt[li];
        if (c > 0) atomicAdd(size + root[li], c);
    }
}

// For each root: its join target (itself unless small).
__global__ __launch_bounds__(kBlock) void ccl_join_kernel(int n, int w, long long S2,
                                                          int min_segment,
                                                          const int* __restrict__ comp,
                                                          const int* __restrict__ size,
                                                          int* __restrict__ join) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    if (comp[r] != r) return;
    const int sz = size[r];
    const bool small = min_segment > 0 ? sz < min_segment : 4ll * sz < S2;
    int j = r;
    if (r != 0 && small) j = comp[(r % w) > 0 ? r - 1 : r - w];
    join[r] = j;
}

// For each root: the root of its join tree; flag[r] = 1 for surviving roots.
__global__ __launch_bounds__(kBlock) void ccl_resolve_kernel(int n, const int* __restrict__ comp,
                                                             const int* __restrict__ join,
                                                             int* __restrict__ fin,
                                                             int* __restrict__ flag) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    if (comp[r] != r) {
        flag[r] = 0;
        return;
    }
    int f = r;
    int j = join[f];
    while (j != f) {
        f = j;
        j = join[f];
    }
    fin[r] = f;
    flag[r] = f == r ? 1 : 0;
}

// Exclusive prefix sum, pass 1: per tile of kScanTile elements, in place,
// and the tile's total.
__global__ __launch_bounds__(kBlock) void scan_tiles_kernel(int n, int* __restrict__ v,
                                                            int* __restrict__ tile_total) {
    __shared__ int s[kBlock];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int item[kScanItems];
    int run = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        item[j] = base + j < n ? v[base + j] : 0;
        const int t = item[j];
        item[j] = run;
        run += t;
    }
    s[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {  // Hillis-Steele inclusive scan
        const int add = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    const int excl = threadIdx.x > 0 ? s[threadIdx.x - 1] : 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) v[base + j] = item[j] + excl;
    if (threadIdx.x == kBlock - 1) tile_total[blockIdx.x] = s[kBlock - 1];
}

// Pass 2 (one workgroup): exclusive scan of the tile totals; the grand total
// goes to *count (if given).
__global__ __launch_bounds__(kBlock) void scan_totals_kernel(int ntiles, int* __restrict__ t,
                                                             int* __restrict__ count) {
    __shared__ int s[kBlock];
    int carry = 0;
    for (int base = 0; base < ntiles; base += kBlock) {
        const int i = base + threadIdx.x;
        const int v = i < ntiles ? t[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const int add = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < ntiles) t[i] = carry + s[threadIdx.x] - v;
        carry += s[kBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0 && count) *count = carry;
}

// Final labels: rank of the pixel's surviving root.
__global__ __launch_bounds__(kBlock) void ccl_relabel_kernel(int n, const int* __restrict__ comp,
                                                             const int* __restrict__ fin,
                                                             const int* __restrict__ rank,
                                                             const int* __restrict__ tile_off,
                                                             int32_t* __restrict__ out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int f = fin[comp[i]];
    out[i] = rank[f] + tile_off[f / kScanTile];
}

}  // namespace

int scan_tiles_for(int n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_connectivity(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                               int32_t min_segment, int32_t* labels_out, int32_t* n_segments,
                               hipStream_t s) {
    const int n = w * h;
    const int nb = (n + kBlock - 1) / kBlock;
    int* comp = ws.ccl0;
    int* size_fin = ws.ccl1;  // sizes, then the resolved join roots
    int* join = ws.ccl2;
    int* rank = ws.ccl3;      // local roots, then surviving-root flags, then their ranks
    hipError_t e;
#define SLIC_STEP(name, ...)                                 \
    do {                                                     \
        KernelTimer t_(name, s);                             \
        __VA_ARGS__;                                         \
        if ((e = hipGetLastError()) != hipSuccess) return e; \
    } while (0)
    const dim3 tiles((w + kTile - 1) / kTile, (h + kTile - 1) / kTile);
    SLIC_STEP("ccl_local",
              ccl_local_kernel<<<tiles, kBlock, 0, s>>>(ws.labels, w, h, comp, rank, size_fin));
    SLIC_STEP("ccl_border", ccl_border_kernel<<<tiles, 2 * kTile, 0, s>>>(ws.labels, w, h, comp));
    SLIC_STEP("ccl_flatten",
              ccl_flatten_kernel<<<tiles, kBlock, 0, s>>>(w, h, comp, rank, size_fin));
    SLIC_STEP("ccl_join",
              ccl_join_kernel<<<nb, kBlock, 0, s>>>(n, w, static_cast<long long>(g.S) * g.S,
                                                    min_segment, comp, size_fin, join));
    // the resolved roots overwrite the sizes, which are no longer needed
    SLIC_STEP("ccl_resolve",
              ccl_resolve_kernel<<<nb, kBlock, 0, s>>>(n, comp, join, size_fin, rank));
    const int ntiles = scan_tiles_for(n);
    SLIC_STEP("ccl_scan", scan_tiles_kernel<<<ntiles, kBlock, 0, s>>>(n, rank, ws.scan));
    SLIC_STEP("ccl_scan", scan_totals_kernel<<<1, kBlock, 0, s>>>(ntiles, ws.scan, n_segments));
    SLIC_STEP("ccl_relabel",
              ccl_relabel_kernel<<<nb, kBlock, 0, s>>>(n, comp, size_fin, rank, ws.scan,
                                                       labels_out));
#undef SLIC_STEP
    return hipSuccess;
}

}  // namespace slic
