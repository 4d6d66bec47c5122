// Finding the cluster associations (Section 3) fused with both halves of
// updating the cluster centres, plus the energy.
//
// Association: each pixel takes the nearest of the (at most nine) centres of
// its own grid cell and the eight neighbouring cells under Eq. 1,
//   D_s = sqrt(dl^2 + da^2 + db^2) + (m/S) sqrt(dx^2 + dy^2),
// whose reference value is evaluated in FP32 in exactly this order, without
// contraction, with correctly rounded square roots; candidates are visited in
// increasing cluster index and replaced only on a strictly smaller distance,
// so ties go to the lowest index.
//
// Certified fast path.  The kernel first evaluates every candidate with fused
// multiply-adds and the hardware square root.  It tracks the smallest and
// second smallest value as integer keys: the distance's bit pattern (a
// non-negative float orders like its bits) with the low four bits replaced
// by the candidate number, so one integer min and one median-of-three keep
// both, and the smallest key names the candidate (lowest index first).  Each
// fast value is within 11 u of the exact real distance and each reference
// value within 4 u (u = 2^-24; relative, all terms are non-negative); the
// keys drop at most 2^-19 relative.  So if the best key's distance is below
// the second's by more than 2^-17 of the latter, the reference argmin is the
// same candidate and no reference value ties with it.  Otherwise (near ties)
// the pixel recomputes every candidate with the reference sequence.
//
// Update, accumulation half: the pixel's colour enters its cluster's sums as
// the exact integer rint(v * 2^18); x and y are integers.  A thread merges
// runs of equal labels among its pixels, adds them to per-workgroup LDS bins
// (int64 atomics), and the workgroup adds its non-empty bins to the global
// int64 sums: exact, so independent of scheduling.
//
// Update, mean half: folded into the next association launch.  Launch t
// accumulates into sums[t % 3], derives the centres it uses from
// sums[(t - 1) % 3] (mean = FP64 quotient of the exact sum by the count,
// colour scaled back by 2^-18, rounded to FP32; a centre with no pixels keeps
// its value), and clears sums[(t + 1) % 3] for the next launch.  The
// workgroup holding a cell's first pixel owns that centre: it stores the new
// centre and count and clears the next buffer.
#include "ccl_tile.h"
#include "slic_internal.h"

#pragma clang fp contract(off)

namespace slic {
namespace {

constexpr int kThreads = 256;
constexpr float kCertify = 0x1p-17f;

// Reference Eq. 1 distance: the exact operation sequence of the definition.
__device__ __forceinline__ float eq1_reference(float cl, float ca, float cb, float cx, float cy,
                                               float l, float a, float b, float xf, float yf,
                                               float wgt) {
    const float dl = cl - l, da = ca - a, db = cb - b;
    float s = dl * dl;
    s = s + da * da;
    s = s + db * db;
    const float dlab = sqrtf(s);
    const float dx = cx - xf, dy = cy - yf;
    float t = dx * dx;
    t = t + dy * dy;
    const float dxy = sqrtf(t);
    const float sp = wgt * dxy;
    return dlab + sp;
}

// Fast Eq. 1 distance (fused multiply-adds, hardware square root); dy2 is
// the squared vertical offset, shared by the pixels of a row.
__device__ __forceinline__ float eq1_fast(float cl, float ca, float cb, float cx, float dy2,
                                          float l, float a, float b, float xf, float wgt) {
    const float dl = cl - l, da = ca - a, db = cb - b;
    const float s = __builtin_fmaf(db, db, __builtin_fmaf(da, da, dl * dl));
    const float dx = cx - xf;
    const float t = __builtin_fmaf(dx, dx, dy2);
    return __builtin_fmaf(wgt, __builtin_amdgcn_sqrtf(t), __builtin_amdgcn_sqrtf(s));
}

// Global (device) memory as a named address space: accesses through such
// pointers compile to global rather than flat memory instructions (flat ones
// also count against the LDS wait counter, so every LDS wait would wait for
// them too).
template <class T>
using gmem = __attribute__((address_space(1))) T;

template <class T>
__device__ __forceinline__ gmem<T>* as_global(T* p) {
    return (gmem<T>*)p;
}

// 16-byte global accesses (builtin vector types: HIP's float4 and int4 are
// classes whose members assume generic pointers).
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef int vi4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load_f4(gmem<const float>* p) {
    const vf4 v = *reinterpret_cast<gmem<const vf4>*>(p);
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void store_f4(gmem<float>* p, float4 v) {
    *reinterpret_cast<gmem<vf4>*>(p) = vf4{v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ void store_i4(gmem<int32_t>* p, int a, int b, int c, int d) {
    *reinterpret_cast<gmem<vi4>*>(p) = vi4{a, b, c, d};
}

typedef float vf2 __attribute__((ext_vector_type(2)));
typedef int vi2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ vf2 load_f2(gmem<const float>* p) {
    return *reinterpret_cast<gmem<const vf2>*>(p);
}

__device__ __forceinline__ void store_i2(gmem<int32_t>* p, int a, int b) {
    *reinterpret_cast<gmem<vi2>*>(p) = vi2{a, b};
}

// Reference argmin over the nine candidates of one pixel (near ties only).
// A cell outside the grid is staged with an infinite colour distance and
// every distance of a cell inside it is finite (the compactness bound), so
// the strict test below never selects an outside cell; the pixel's own cell
// (slot 4) is the starting choice.
__device__ __forceinline__ int reference_slot(const float4* cen4, const float* ceny, int base,
                                              int ncx, float l, float a, float b, float xf,
                                              float yf, float wgt) {
    float bref = __builtin_huge_valf();
    int sref = 4;
#pragma unroll 1
    for (int c = 0; c < 9; ++c) {
        const int li = base + (c / 3) * ncx + (c % 3);
        const float4 q = cen4[li];
        const float d = eq1_reference(q.x, q.y, q.z, q.w, ceny[li], l, a, b, xf, yf, wgt);
        if (d < bref) {
            bref = d;
            sref = c;
        }
    }
    return sref;
}

// A workgroup's image: from the kernel argument (one image) or, for a batch,
// from the image table through the tile-to-image map.
template <bool kBatch>
__device__ __forceinline__ void resolve_image(const AssignImage& single, const AssignTileMap& map,
                                              AssignImage* g, int* bx, int* by) {
    if constexpr (kBatch) {
        const int img = map.tile_image[blockIdx.x];
        *g = map.images[img];
        const int local = static_cast<int>(blockIdx.x) - map.tile_first[img];
        *bx = local % g->tiles_x;
        *by = local / g->tiles_x;
    } else {
        *g = single;
        *bx = blockIdx.x;
        *by = blockIdx.y;
    }
}

// Shared-memory layout (dynamic): for every cell of the staged window
// (the workgroup's cells plus a one-cell ring, out-of-grid cells included):
//   float4 cen4[n] (L, a, b, x), float ceny[n], int kidx[n] (-1: none),
//   u64 bins[4][n] (sum qL, sum qa, sum qb, packed x'|y'<<20|count<<40).
__host__ __device__ inline size_t assign_lds_bytes(int ncells) {
    return static_cast<size_t>(ncells) * (16 + 4 + 4 + 32) + 16;
}

// Launch shape of a variant: each thread owns VEC horizontally adjacent
// pixels in each of ROWS consecutive rows.  VEC = 2 or 4 uses 8- or 16-byte
// loads and evaluates each staged centre once for the VEC pixels, so it
// needs them in one cell (S % VEC == 0) and aligned rows (width % VEC == 0).
template <int VEC, int ROWS, int TX = (VEC == 4 ? 16 : 32)>
struct Shape {
    static constexpr int kTX = TX;  // threads per row
    static constexpr int kTY = kThreads / kTX;
    static constexpr int kTileW = kTX * VEC;
    static constexpr int kTileH = kTY * ROWS;
    static constexpr int kPx = VEC * ROWS;
};

__device__ __forceinline__ void add_bin(unsigned long long* bins, int ncells, int cell,
                                        long long rl, long long ra, long long rb,
                                        unsigned long long rxyc) {
    atomicAdd(bins + cell, static_cast<unsigned long long>(rl));
    atomicAdd(bins + ncells + cell, static_cast<unsigned long long>(ra));
    atomicAdd(bins + 2 * ncells + cell, static_cast<unsigned long long>(rb));
    atomicAdd(bins + 3 * ncells + cell, rxyc);
}

// The squared-sum distance of the SLIC paper the method builds on (an
// option): d_lab^2 + w^2 d_xy^2 in FP32 in this order, no square roots, so
// its argmin is taken exactly.
__device__ __forceinline__ float dist_squared(float cl, float ca, float cb, float cx, float dy2,
                                              float l, float a, float b, float xf, float wgt) {
    const float dl = cl - l, da = ca - a, db = cb - b;
    float s = dl * dl;
    s = s + da * da;
    s = s + db * db;
    const float dx = cx - xf;
    float t = dx * dx;
    t = t + dy2;
    const float w2 = wgt * wgt;
    const float sp = w2 * t;
    return s + sp;
}

// Launch modes: one image, one image with the convergence stop, a batch,
// and one image whose launch is the last before the connectivity clean-up
// and also finds the tile-local components of its labels (32 x 32 tiles
// only).  Each is its own instantiation, so a kernel reads only the
// arguments its mode uses and takes no branch on them on the way in.
enum AssignMode { kModeSingle = 0, kModeConverge = 1, kModeBatch = 2, kModeFinalCcl = 3 };

// Outputs of the tile-local connectivity step (kModeFinalCcl): every
// pixel's local root as a global index and as an index inside its tile, and
// the local roots' part sizes.
struct AssignCcl {
    int32_t* comp;
    int32_t* lroot;
    int32_t* size;
};

// A launch's shape: its variant's, except that the final launch with the
// tile-local components has the connectivity pass's 32 x 32 tiles.
template <int VEC, int ROWS, int MODE>
using LaunchShape =
    Shape<VEC, ROWS, MODE == kModeFinalCcl ? tile_ccl::kTile / VEC : (VEC == 4 ? 16 : 32)>;

// The Eq. 1 variants are held to 128 VGPRs (four waves per SIMD), which
// they need for latency hiding at large frames.
template <int VEC, int ROWS, int DIST, int MODE>
__global__ __launch_bounds__(kThreads, DIST == 0 ? 4 : 1) void assign_kernel(
    AssignImage single, AssignTileMap map, long long t, Converge cv, AssignCcl cc,
    int store_labels) {
    using Sh = LaunchShape<VEC, ROWS, MODE>;
    constexpr bool kConv = MODE == kModeConverge;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long s_shift;
    if constexpr (kConv) {  // convergence stop: every workgroup takes the same decision
        if (cv.ctl[3] != 0) return;
        if (t > cv.t_first && cv.ctl[(t - 1) % 3] < cv.limit) {
            if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
                cv.ctl[3] = 1;
                cv.ctl[4] = t - cv.t_first;
            }
            return;
        }
        if (threadIdx.x == 0) {
            s_shift = 0ull;
            if (blockIdx.x == 0 && blockIdx.y == 0) cv.ctl[(t + 1) % 3] = 0;
        }
    }
    long long my_shift = 0;
    AssignImage g;
    int bx, by;
    resolve_image<MODE == kModeBatch>(single, map, &g, &bx, &by);
    const size_t ring = static_cast<size_t>(g.K) * kSumStride;
    gmem<long long>* const sums = as_global(g.sums);
    gmem<long long>* const sums_acc = sums + ring * static_cast<size_t>(t % 3);
    gmem<const long long>* const sums_prev =
        t > 0 ? sums + ring * static_cast<size_t>((t + 2) % 3) : nullptr;
    gmem<long long>* const sums_next = sums + ring * static_cast<size_t>((t + 1) % 3);
    gmem<float>* const cen = as_global(g.cen);
    gmem<int32_t>* const labels = as_global(g.labels);
    const int x0 = bx * Sh::kTileW, y0 = by * Sh::kTileH;
    const int tx = threadIdx.x % Sh::kTX, ty = threadIdx.x / Sh::kTX;
    const int x = x0 + tx * VEC;
    const bool col_ok = x < g.w;

    const int S = g.S;
    const int gx_lo = x0 / S - 1, gy_lo = y0 / S - 1;
    const int gx_hi = (min(x0 + Sh::kTileW, g.w) - 1) / S + 1;
    const int gy_hi = (min(y0 + Sh::kTileH, g.h) - 1) / S + 1;
    const int ncx = gx_hi - gx_lo + 1, ncy = gy_hi - gy_lo + 1, ncells = ncx * ncy;
    float4* cen4 = reinterpret_cast<float4*>(smem);
    float* ceny = reinterpret_cast<float*>(cen4 + ncells);
    int* kidx = reinterpret_cast<int*>(ceny + ncells);
    // 24 * ncells bytes precede the bins, a multiple of 8; offsets from smem
    // keep the bins' LDS address space visible to the compiler, so their
    // atomics are LDS atomics rather than flat ones
    unsigned long long* bins =
        reinterpret_cast<unsigned long long*>(smem + static_cast<size_t>(ncells) * 24);

    // ---- staging of the candidate centres, in two halves: the loads of a
    // window cell (the centre the previous launch used and, from the second
    // launch on, the previous launch's sums), then the means, the owner's
    // stores and the LDS entries.  The loads are branch-free, from a clamped
    // cell: a branch around them would make their first use, and hence the
    // wait for them, come early.
    struct Slot {
        float4 old4;
        float oldy;
        long long sv[kSumStride];
        int k;       // cluster, -1: past the window or outside the grid
        int cx, cy;  // its grid cell
    };
    gmem<const long long>* const sums_src = sums_prev ? sums_prev : sums_acc;
    // row of window cell i: floor((i + 1/2) / ncx) through the hardware
    // reciprocal; for i < 4096 and ncx <= 64 the product is within 2^-10 of
    // the quotient, which lies at least 1/128 from an integer, so the floor
    // is exact
    const float inv_ncx = __builtin_amdgcn_rcpf(static_cast<float>(ncx));
    auto stage_load = [&](int i) {
        Slot st;
        const int row = static_cast<int>((static_cast<float>(i) + 0.5f) * inv_ncx);
        const int cx = gx_lo + (i - row * ncx), cy = gy_lo + row;
        st.cx = cx;
        st.cy = cy;
        const bool live = i < ncells && cx >= 0 && cy >= 0 && cx < g.ns_c && cy < g.ns_r;
        st.k = live ? cy * g.ns_c + cx : -1;
        const int kk = live ? st.k : 0;
        gmem<float>* c = cen + static_cast<size_t>(kk) * kCenStride;
        st.old4 = load_f4(c);
        st.oldy = c[4];
        gmem<const long long>* sp = sums_src + static_cast<size_t>(kk) * kSumStride;
#pragma unroll
        for (int j = 0; j < kSumStride; ++j) st.sv[j] = sp[j];
        return st;
    };
    // the previous launch's means (an empty cluster keeps its centre); the
    // owner stores the new centre and count (and the convergence shift)
    auto update_centre = [&](const long long* sv, float4 old4, float oldy, bool owner,
                             gmem<float>* c, int k, float4* vout, float* vyout) {
        // the means are computed unconditionally (and selected), so the
        // sums' loads are not deferred behind a test of the count
        const long long n = sv[5];
        const double dn = static_cast<double>(n > 0 ? n : 1);
        const double inv = 1.0 / static_cast<double>(1 << kQShift);
        const double ml = static_cast<double>(sv[0]) / dn;
        const double ma = static_cast<double>(sv[1]) / dn;
        const double mb = static_cast<double>(sv[2]) / dn;
        const float4 m4 = make_float4(static_cast<float>(ml * inv), static_cast<float>(ma * inv),
                                      static_cast<float>(mb * inv),
                                      static_cast<float>(static_cast<double>(sv[3]) / dn));
        const float my = static_cast<float>(static_cast<double>(sv[4]) / dn);
        const bool moved = n > 0;
        const float4 v = make_float4(moved ? m4.x : old4.x, moved ? m4.y : old4.y,
                                     moved ? m4.z : old4.z, moved ? m4.w : old4.w);
        const float vy = moved ? my : oldy;
        if (owner && moved) {
            if constexpr (kConv) {  // L1 shift, each component rint(|d| 2^18)
                const double q = static_cast<double>(1 << kQShift);
                my_shift += llrint(fabs(static_cast<double>(v.x) - old4.x) * q) +
                            llrint(fabs(static_cast<double>(v.y) - old4.y) * q) +
                            llrint(fabs(static_cast<double>(v.z) - old4.z) * q) +
                            llrint(fabs(static_cast<double>(v.w) - old4.w) * q) +
                            llrint(fabs(static_cast<double>(vy) - oldy) * q);
            }
            store_f4(c, v);
            c[4] = vy;
        }
        if (owner) as_global(g.counts)[k] = static_cast<int32_t>(n);
        *vout = v;
        *vyout = vy;
    };
    auto stage_finish = [&](int i, const Slot& st) {
        if (i >= ncells) return;
        const int cx = st.cx, cy = st.cy;
        for (int j = 0; j < 4; ++j) bins[j * ncells + i] = 0ull;
        if (st.k < 0) {
            // no centre here: an infinite colour distance never wins
            cen4[i] = make_float4(__builtin_huge_valf(), 0.0f, 0.0f, 0.0f);
            ceny[i] = 0.0f;
            kidx[i] = -1;
            return;
        }
        const int k = st.k;
        kidx[i] = k;
        const bool owner = (cx * S) / Sh::kTileW == bx && (cy * S) / Sh::kTileH == by;
        gmem<float>* c = cen + static_cast<size_t>(k) * kCenStride;
        const float4 old4 = st.old4;  // the centre the previous launch used
        const float oldy = st.oldy;
        float4 v = old4;
        float vy = oldy;
        if (sums_prev) update_centre(st.sv, old4, oldy, owner, c, k, &v, &vy);
        if (owner) {
            gmem<long long>* z = sums_next + static_cast<size_t>(k) * kSumStride;
            for (int j = 0; j < kSumStride; ++j) z[j] = 0;
        }
        cen4[i] = v;
        ceny[i] = vy;
    };

    // Variants with several rows per thread (large frames, where every
    // workgroup of a launch is resident at once) load the thread's first cell
    // before its pixels: a wave's loads return in order, so the staging and
    // the barrier after it wait only for the centres while the pixel data is
    // still arriving.  One-row variants (small frames, mostly one wave per
    // SIMD) load the pixels first and only the cells they hold: there the
    // loads of the waves without a cell would delay their pixels.
    constexpr bool kStageFirst = ROWS >= 2;
    Slot first;
    first.k = -1;
    if constexpr (kStageFirst) {
        first = stage_load(threadIdx.x);
        __builtin_amdgcn_sched_barrier(0);  // keep the pixel loads after these
    }

    // ---- prefetch this thread's pixels (they do not depend on the centres).
    // Every lane loads (pixels outside the image read a clamped position and
    // are then zeroed), so the loads are issued unconditionally.
    float pl[ROWS][VEC], pa[ROWS][VEC], pb[ROWS][VEC];
    {
        gmem<const float>* const Lg = as_global(g.L);
        gmem<const float>* const Ag = as_global(g.A);
        gmem<const float>* const Bg = as_global(g.B);
        const int xc = min(x, g.w - VEC);  // VEC > 1 needs width % VEC == 0
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = y0 + ty * ROWS + r;
            const bool in = col_ok && y < g.h;
            const size_t pi = static_cast<size_t>(min(y, g.h - 1)) * g.w + xc;
            if constexpr (VEC == 4) {
                const float4 l4 = load_f4(Lg + pi);
                const float4 a4 = load_f4(Ag + pi);
                const float4 b4 = load_f4(Bg + pi);
                pl[r][0] = l4.x; pl[r][1] = l4.y; pl[r][2] = l4.z; pl[r][3] = l4.w;
                pa[r][0] = a4.x; pa[r][1] = a4.y; pa[r][2] = a4.z; pa[r][3] = a4.w;
                pb[r][0] = b4.x; pb[r][1] = b4.y; pb[r][2] = b4.z; pb[r][3] = b4.w;
            } else if constexpr (VEC == 2) {
                const vf2 l2 = load_f2(Lg + pi), a2 = load_f2(Ag + pi), b2 = load_f2(Bg + pi);
                pl[r][0] = l2.x; pl[r][1] = l2.y;
                pa[r][0] = a2.x; pa[r][1] = a2.y;
                pb[r][0] = b2.x; pb[r][1] = b2.y;
            } else {
                pl[r][0] = Lg[pi];
                pa[r][0] = Ag[pi];
                pb[r][0] = Bg[pi];
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                pl[r][v] = in ? pl[r][v] : 0.0f;
                pa[r][v] = in ? pa[r][v] : 0.0f;
                pb[r][v] = in ? pb[r][v] : 0.0f;
            }
        }
    }

    if constexpr (kStageFirst) {
        stage_finish(threadIdx.x, first);
        for (int i = threadIdx.x + kThreads; i < ncells; i += kThreads)
            stage_finish(i, stage_load(i));
    } else {
        // one loop, each cell's loads and means together (the compiler then
        // overlaps the five FP64 divisions of a cell)
        for (int i = threadIdx.x; i < ncells; i += kThreads) {
            const int cx = gx_lo + i % ncx, cy = gy_lo + i / ncx;
            for (int j = 0; j < 4; ++j) bins[j * ncells + i] = 0ull;
            if (cx < 0 || cy < 0 || cx >= g.ns_c || cy >= g.ns_r) {
                // no centre here: an infinite colour distance never wins
                cen4[i] = make_float4(__builtin_huge_valf(), 0.0f, 0.0f, 0.0f);
                ceny[i] = 0.0f;
                kidx[i] = -1;
                continue;
            }
            const int k = cy * g.ns_c + cx;
            kidx[i] = k;
            const bool owner = (cx * S) / Sh::kTileW == bx && (cy * S) / Sh::kTileH == by;
            gmem<float>* c = cen + static_cast<size_t>(k) * kCenStride;
            // every load first, so that one memory round trip serves them all
            const float4 old4 = load_f4(c);  // the centre the previous launch used
            const float oldy = c[4];
            long long sv[kSumStride] = {};
            if (sums_prev) {
                gmem<const long long>* sp = sums_prev + static_cast<size_t>(k) * kSumStride;
#pragma unroll
                for (int j = 0; j < kSumStride; ++j) sv[j] = sp[j];
            }
            float4 v = old4;
            float vy = oldy;
            if (sums_prev) update_centre(sv, old4, oldy, owner, c, k, &v, &vy);
            if (owner) {
                gmem<long long>* z = sums_next + static_cast<size_t>(k) * kSumStride;
                for (int j = 0; j < kSumStride; ++j) z[j] = 0;
            }
            cen4[i] = v;
            ceny[i] = vy;
        }
    }
    __syncthreads();
    if (my_shift) atomicAdd(&s_shift, static_cast<unsigned long long>(my_shift));

    // ---- associate: fast distances for every candidate, shared by the VEC
    // pixels of a row (they lie in one cell)
    // window column of the left candidates (columns past the image edge use the
    // tile's first cell, so every staged-window index stays in range)
    const int gx_rel = (col_ok ? x / S : x0 / S) - gx_lo - 1;
    int cellv[ROWS][VEC];
    unsigned need = 0;  // pixels whose fast argmin is not certified: bit r * VEC + v
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + ty * ROWS + r;
        const float yf = static_cast<float>(y);
        const int base = (min(y, g.h - 1) / S - gy_lo - 1) * ncx + gx_rel;
        if constexpr (DIST == 1) {
            // exact: (distance bits, slot) as one 64-bit key, lowest slot on ties
            unsigned long long bk[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) bk[v] = ~0ull;
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const int li = base + (c / 3) * ncx + (c % 3);
                const float4 q = cen4[li];
                const float dy = ceny[li] - yf;
                const float dy2 = dy * dy;
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const float d = dist_squared(q.x, q.y, q.z, q.w, dy2, pl[r][v], pa[r][v],
                                                 pb[r][v], static_cast<float>(x + v), g.wgt);
                    const unsigned long long key =
                        (static_cast<unsigned long long>(__float_as_uint(d)) << 4) |
                        static_cast<unsigned long long>(c);
                    bk[v] = key < bk[v] ? key : bk[v];
                }
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                // an out-of-grid cell (infinite distance) can only come first
                // when no distance is finite; the own cell is then taken
                int slot = static_cast<int>(bk[v] & 15ull);
                const int cell = base + (slot / 3) * ncx + (slot % 3);
                cellv[r][v] = kidx[cell] < 0 ? base + ncx + 1 : cell;
            }
            continue;
        }
        unsigned best[VEC], second[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) best[v] = second[v] = 0xFFFFFFFFu;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const int li = base + (c / 3) * ncx + (c % 3);
            const float4 q = cen4[li];
            const float dy = ceny[li] - yf;
            const float dy2 = dy * dy;
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const float d = eq1_fast(q.x, q.y, q.z, q.w, dy2, pl[r][v], pa[r][v], pb[r][v],
                                         static_cast<float>(x + v), g.wgt);
                const unsigned key = (__float_as_uint(d) & ~15u) | static_cast<unsigned>(c);
                // median of (best, second, key) given best <= second
                second[v] = max(best[v], min(second[v], key));
                best[v] = min(best[v], key);
            }
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int slot = static_cast<int>(best[v] & 15u);
            const float bf = __uint_as_float(best[v] & ~15u);
            const float sf = __uint_as_float(second[v] & ~15u);
            if (!(bf < __builtin_fmaf(sf, -kCertify, sf))) need |= 1u << (r * VEC + v);
            cellv[r][v] = base + (slot / 3) * ncx + (slot % 3);
        }
    }
    // near ties (a few pixels per frame): the reference argmin, after the
    // fast pass, whose keys are then dead, and inline (a call would pin the
    // fast pass's live values to the callee-saved registers)
    if (need) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = y0 + ty * ROWS + r;
            const int base = (min(y, g.h - 1) / S - gy_lo - 1) * ncx + gx_rel;
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                if (!(need & (1u << (r * VEC + v)))) continue;
                const int slot = reference_slot(cen4, ceny, base, ncx, pl[r][v], pa[r][v],
                                                pb[r][v], static_cast<float>(x + v),
                                                static_cast<float>(y), g.wgt);
                cellv[r][v] = base + (slot / 3) * ncx + (slot % 3);
            }
        }
    }

    // ---- labels, then runs of equal cells into the LDS bins (the last
    // launch before the connectivity clean-up only stores the labels: no
    // update follows it)
    constexpr bool kSums = MODE != kModeFinalCcl;
    const float scale = static_cast<float>(1 << kQShift);
    int run_cell = -1;
    int rl = 0, ra = 0, rb = 0;
    unsigned long long rxyc = 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + ty * ROWS + r;
        if (!col_ok || y >= g.h) continue;
        const size_t pi = static_cast<size_t>(y) * g.w + x;
        if (store_labels) {
            if constexpr (VEC == 4) {
                store_i4(labels + pi, kidx[cellv[r][0]], kidx[cellv[r][1]], kidx[cellv[r][2]],
                         kidx[cellv[r][3]]);
            } else if constexpr (VEC == 2) {
                store_i2(labels + pi, kidx[cellv[r][0]], kidx[cellv[r][1]]);
            } else {
                labels[pi] = kidx[cellv[r][0]];
            }
        }
        if constexpr (!kSums) continue;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int cell = cellv[r][v];
            const int ql = static_cast<int>(rintf(pl[r][v] * scale));
            const int qa = static_cast<int>(rintf(pa[r][v] * scale));
            const int qb = static_cast<int>(rintf(pb[r][v] * scale));
            const unsigned long long xyc = static_cast<unsigned long long>(x + v - x0) |
                                           (static_cast<unsigned long long>(y - y0) << 20) |
                                           (1ull << 40);
            if (cell != run_cell) {
                if (run_cell >= 0) add_bin(bins, ncells, run_cell, rl, ra, rb, rxyc);
                run_cell = cell;
                rl = ql;
                ra = qa;
                rb = qb;
                rxyc = xyc;
            } else {
                rl += ql;
                ra += qa;
                rb += qb;
                rxyc += xyc;
            }
        }
    }
    if constexpr (kSums) {
        if (run_cell >= 0) add_bin(bins, ncells, run_cell, rl, ra, rb, rxyc);
        __syncthreads();
        if constexpr (kConv) {
            if (threadIdx.x == 0 && s_shift)
                atomicAdd(reinterpret_cast<unsigned long long*>(cv.ctl + t % 3), s_shift);
        }

        // ---- add the workgroup's bins to the global sums
        for (int i = threadIdx.x; i < ncells; i += kThreads) {
            const unsigned long long p = bins[3 * ncells + i];
            const long long n = static_cast<long long>(p >> 40);
            if (n == 0) continue;
            const long long sx = static_cast<long long>(p & 0xFFFFFull) + n * x0;
            const long long sy = static_cast<long long>((p >> 20) & 0xFFFFFull) + n * y0;
            gmem<unsigned long long>* s = reinterpret_cast<gmem<unsigned long long>*>(
                sums_acc + static_cast<size_t>(kidx[i]) * kSumStride);
            const unsigned long long add[kSumStride] = {
                bins[i], bins[ncells + i], bins[2 * ncells + i],
                static_cast<unsigned long long>(sx), static_cast<unsigned long long>(sy),
                static_cast<unsigned long long>(n)};
#pragma unroll
            for (int j = 0; j < kSumStride; ++j)
                __hip_atomic_fetch_add(s + j, add[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // ---- the tile-local components of the labels just written (the
    // connectivity pass's first step, on the same 32 x 32 tile)
    if constexpr (MODE == kModeFinalCcl) {
        static_assert(Sh::kTileW == tile_ccl::kTile && Sh::kTileH == tile_ccl::kTile &&
                          kThreads == tile_ccl::kBlock,
                      "the tile-local components need the 32 x 32 connectivity tile");
        __shared__ int clab[tile_ccl::kTilePx];
        __shared__ int cpar[tile_ccl::kTilePx];
        __shared__ int ccnt[tile_ccl::kTilePx];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = y0 + ty * ROWS + r;
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                clab[(ty * ROWS + r) * tile_ccl::kTile + tx * VEC + v] =
                    col_ok && y < g.h ? kidx[cellv[r][v]] : -1;
        }
#pragma unroll
        for (int j = 0; j < tile_ccl::kPxPerThread; ++j)
            ccnt[threadIdx.x + j * tile_ccl::kBlock] = 0;
        __syncthreads();
        tile_ccl::tile_components(clab, cpar, ccnt, x0, y0, g.w, g.h, as_global(cc.comp),
                                  as_global(cc.lroot), as_global(cc.size));
    }
}

__global__ void converge_reset_kernel(long long* ctl) {
    if (threadIdx.x < 8) ctl[threadIdx.x] = 0;
}

__global__ void converge_result_kernel(const long long* ctl, int max_iters, int32_t* out) {
    if (threadIdx.x == 0) *out = ctl[3] ? static_cast<int32_t>(ctl[4]) : max_iters;
}

constexpr int kEnergyBlock = 256;

__global__ __launch_bounds__(kEnergyBlock) void energy_kernel(
    const float* __restrict__ L, const float* __restrict__ A, const float* __restrict__ B, int w,
    int n, float wgt, int dist, const float* __restrict__ cen, const int32_t* __restrict__ labels,
    double* __restrict__ partial) {
    __shared__ double red[kEnergyBlock];
    const int i = blockIdx.x * kEnergyBlock + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const float* c = cen + static_cast<size_t>(labels[i]) * kCenStride;
        const float xf = static_cast<float>(i % w), yf = static_cast<float>(i / w);
        if (dist) {
            const float dy = c[4] - yf;
            v = static_cast<double>(
                sqrtf(dist_squared(c[0], c[1], c[2], c[3], dy * dy, L[i], A[i], B[i], xf, wgt)));
        } else {
            v = static_cast<double>(eq1_reference(c[0], c[1], c[2], c[3], c[4], L[i], A[i], B[i],
                                                  xf, yf, wgt));
        }
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = kEnergyBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kEnergyBlock) void energy_final_kernel(const double* __restrict__ partial,
                                                                    int nblocks, double n_pixels,
                                                                    double* __restrict__ out) {
    __shared__ double red[kEnergyBlock];
    double v = 0.0;
    for (int j = threadIdx.x; j < nblocks; j += kEnergyBlock) v = v + partial[j];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = kEnergyBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / n_pixels;
}

__global__ __launch_bounds__(256) void export_centres_kernel(int K, const float* __restrict__ cen,
                                                             const int32_t* __restrict__ counts,
                                                             float* __restrict__ out,
                                                             int32_t* __restrict__ out_counts) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    for (int j = 0; j < 5; ++j)
        out[5 * static_cast<size_t>(k) + j] = cen[static_cast<size_t>(k) * kCenStride + j];
    if (out_counts) out_counts[k] = counts[k];
}

__global__ __launch_bounds__(256) void import_centres_kernel(int K, const float* __restrict__ in,
                                                             float* __restrict__ cen) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    for (int j = 0; j < 5; ++j)
        cen[static_cast<size_t>(k) * kCenStride + j] = in[5 * static_cast<size_t>(k) + j];
}

template <int VEC, int ROWS>
size_t variant_lds(int S) {
    using Sh = Shape<VEC, ROWS>;
    // window of cells over any tile: at most (tile - 1)/S + 4 per side
    return assign_lds_bytes(((Sh::kTileW - 1) / S + 4) * ((Sh::kTileH - 1) / S + 4));
}

template <int VEC, int ROWS, int DIST>
hipError_t launch_variant(const AssignImage& a, const AssignTileMap& map, int total_tiles,
                          int min_S, long long t, const Converge& cv, bool store,
                          hipStream_t s) {
    using Sh = Shape<VEC, ROWS>;
    dim3 grid;
    if (map.images) {
        grid = dim3(total_tiles);
    } else {
        grid = dim3((a.w + Sh::kTileW - 1) / Sh::kTileW, (a.h + Sh::kTileH - 1) / Sh::kTileH);
    }
    KernelTimer timer("assign", s);
    const size_t lds = variant_lds<VEC, ROWS>(min_S);
    if (map.images) {
        assign_kernel<VEC, ROWS, DIST, kModeBatch><<<grid, kThreads, lds, s>>>(a, map, t, cv, {},
                                                                              store);
    } else if (cv.ctl) {
        assign_kernel<VEC, ROWS, DIST, kModeConverge><<<grid, kThreads, lds, s>>>(a, map, t, cv,
                                                                                 {}, store);
    } else {
        assign_kernel<VEC, ROWS, DIST, kModeSingle><<<grid, kThreads, lds, s>>>(a, map, t, cv, {},
                                                                               store);
    }
    return hipGetLastError();
}

// The final launch with the tile-local components, on 32 x 32 tiles: four
// pixels of a row per thread (VEC = 4, eight threads per row) below 1 Mpix
// where the step and the width allow it, else one pixel in each of four
// rows (at 1920 x 1080 the faster of the two, as among the variants).
template <int VEC, int ROWS>
size_t final_ccl_lds(int S) {
    using Sh = LaunchShape<VEC, ROWS, kModeFinalCcl>;
    return assign_lds_bytes(((Sh::kTileW - 1) / S + 4) * ((Sh::kTileH - 1) / S + 4));
}

template <int VEC, int ROWS, int DIST>
hipError_t launch_final_ccl(const AssignImage& a, long long t, const AssignCcl& cc, int S,
                            hipStream_t s) {
    using Sh = LaunchShape<VEC, ROWS, kModeFinalCcl>;
    const dim3 grid((a.w + Sh::kTileW - 1) / Sh::kTileW, (a.h + Sh::kTileH - 1) / Sh::kTileH);
    const AssignTileMap none{nullptr, nullptr, nullptr};
    const Converge off{nullptr, 0, 0};
    KernelTimer timer("assign", s);
    assign_kernel<VEC, ROWS, DIST, kModeFinalCcl><<<grid, kThreads, final_ccl_lds<VEC, ROWS>(S),
                                                     s>>>(a, none, t, off, cc, 1);
    return hipGetLastError();
}

bool final_ccl_vec4(int32_t w, int32_t h, int32_t S) {
    return static_cast<long long>(w) * h < (1ll << 20) && S % 4 == 0 && w % 4 == 0 &&
           final_ccl_lds<4, 1>(S) <= (64u << 10);
}

using LaunchFn = hipError_t (*)(const AssignImage&, const AssignTileMap&, int, int, long long,
                                const Converge&, bool, hipStream_t);

struct VariantDesc {
    int vec, rows;
    size_t (*lds)(int);
    LaunchFn launch[2];  // Eq. 1, squared-sum distance
};

const VariantDesc kVariants[] = {
    {1, 1, variant_lds<1, 1>, {launch_variant<1, 1, 0>, launch_variant<1, 1, 1>}},
    {1, 2, variant_lds<1, 2>, {launch_variant<1, 2, 0>, launch_variant<1, 2, 1>}},
    {1, 4, variant_lds<1, 4>, {launch_variant<1, 4, 0>, launch_variant<1, 4, 1>}},
    {4, 1, variant_lds<4, 1>, {launch_variant<4, 1, 0>, launch_variant<4, 1, 1>}},
    {4, 2, variant_lds<4, 2>, {launch_variant<4, 2, 0>, launch_variant<4, 2, 1>}},
    {2, 1, variant_lds<2, 1>, {launch_variant<2, 1, 0>, launch_variant<2, 1, 1>}},
    {2, 2, variant_lds<2, 2>, {launch_variant<2, 2, 0>, launch_variant<2, 2, 1>}},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

int assign_variant_count() { return kNumVariants; }

bool assign_variant_shape(int variant, int* vec, int* rows, int* tile_w, int* tile_h) {
    if (variant < 1 || variant > kNumVariants) return false;
    const VariantDesc& d = kVariants[variant - 1];
    const int tx = d.vec == 4 ? 16 : 32;
    if (vec) *vec = d.vec;
    if (rows) *rows = d.rows;
    if (tile_w) *tile_w = tx * d.vec;
    if (tile_h) *tile_h = (kThreads / tx) * d.rows;
    return true;
}

bool assign_variant_supported(int variant, int32_t w, int32_t h, int32_t S) {
    (void)h;
    if (variant < 1 || variant > kNumVariants) return false;
    const VariantDesc& d = kVariants[variant - 1];
    if (d.vec > 1 && (S % d.vec != 0 || w % d.vec != 0)) return false;
    return d.lds(S) <= (64u << 10);
}

int assign_default_variant(int32_t w, int32_t h, int32_t S) {
    const long long n = static_cast<long long>(w) * h;
    // small frames are latency bound: many workgroups; larger frames
    // amortise the staged centres over more pixels per thread (the
    // autotuner's picks: 2 at 320x240, 4 at 640x480, 5 at 1920x1080); a
    // shape the step or width does not allow falls back down the table
    int v = 2;
    if (n >= (1ll << 20))
        v = 5;
    else if (n >= (1ll << 17))
        v = 4;
    while (v > 1 && !assign_variant_supported(v, w, h, S)) --v;
    return v;
}

bool assign_tiles(int variant, int32_t w, int32_t h, int* tiles_x, int* tiles_y) {
    int tw = 0, th = 0;
    if (!assign_variant_shape(variant, nullptr, nullptr, &tw, &th)) return false;
    if (tiles_x) *tiles_x = (w + tw - 1) / tw;
    if (tiles_y) *tiles_y = (h + th - 1) / th;
    return true;
}

AssignImage assign_image(const Workspace& ws, int32_t w, int32_t h, const Grid& g, int variant) {
    AssignImage a;
    a.L = ws.L;
    a.A = ws.A;
    a.B = ws.B;
    a.w = w;
    a.h = h;
    a.S = g.S;
    a.ns_c = g.ns_c;
    a.ns_r = g.ns_r;
    a.K = g.K;
    a.wgt = g.w;
    a.cen = ws.cen;
    a.counts = ws.counts;
    a.labels = ws.labels;
    a.sums = ws.sums;
    a.tiles_x = 0;
    assign_tiles(variant, w, h, &a.tiles_x, nullptr);
    return a;
}

hipError_t launch_assign(const Workspace& ws, int32_t w, int32_t h, const Grid& g, int64_t t,
                         int variant, hipStream_t s, const Converge* cv, bool store_labels) {
    if (!assign_variant_supported(variant, w, h, g.S)) variant = assign_default_variant(w, h, g.S);
    const AssignImage a = assign_image(ws, w, h, g, variant);
    const AssignTileMap none{nullptr, nullptr, nullptr};
    const Converge off{nullptr, 0, 0};
    return kVariants[variant - 1].launch[g.dist ? 1 : 0](a, none, 0, g.S, t, cv ? *cv : off,
                                                         store_labels, s);
}

bool assign_final_ccl_supported(int32_t w, int32_t h, int32_t S) {
    (void)w;
    (void)h;
    return final_ccl_lds<1, 4>(S) <= (64u << 10);
}

hipError_t launch_assign_final_ccl(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                                  int64_t t, hipStream_t s) {
    if (!assign_final_ccl_supported(w, h, g.S)) return hipErrorInvalidValue;
    AssignImage a = assign_image(ws, w, h, g, 1);
    a.tiles_x = (w + tile_ccl::kTile - 1) / tile_ccl::kTile;
    const AssignCcl cc{ws.ccl0, ws.ccl3, ws.ccl1};  // as the connectivity pass names them
    if (final_ccl_vec4(w, h, g.S))
        return g.dist ? launch_final_ccl<4, 1, 1>(a, t, cc, g.S, s)
                      : launch_final_ccl<4, 1, 0>(a, t, cc, g.S, s);
    return g.dist ? launch_final_ccl<1, 4, 1>(a, t, cc, g.S, s)
                  : launch_final_ccl<1, 4, 0>(a, t, cc, g.S, s);
}

hipError_t launch_assign_batch(const AssignTileMap& map, int total_tiles, int min_S, int64_t t,
                               int variant, int dist, hipStream_t s, bool store_labels) {
    if (variant < 1 || variant > kNumVariants || !map.images) return hipErrorInvalidValue;
    AssignImage unused{};
    const Converge off{nullptr, 0, 0};
    return kVariants[variant - 1].launch[dist ? 1 : 0](unused, map, total_tiles, min_S, t, off,
                                                       store_labels, s);
}

hipError_t launch_energy(const Workspace& ws, int32_t w, int32_t h, const Grid& g, double* out,
                         hipStream_t s) {
    const int n = w * h;
    const int nb = (n + kEnergyBlock - 1) / kEnergyBlock;
    {
        KernelTimer t("energy", s);
        energy_kernel<<<nb, kEnergyBlock, 0, s>>>(ws.L, ws.A, ws.B, w, n, g.w, g.dist, ws.cen,
                                                  ws.labels, ws.partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    KernelTimer t("energy_final", s);
    energy_final_kernel<<<1, kEnergyBlock, 0, s>>>(ws.partial, nb, static_cast<double>(n), out);
    return hipGetLastError();
}

hipError_t launch_converge_reset(long long* ctl, hipStream_t s) {
    converge_reset_kernel<<<1, 64, 0, s>>>(ctl);
    return hipGetLastError();
}

hipError_t launch_converge_result(const long long* ctl, int32_t max_iters, int32_t* out,
                                  hipStream_t s) {
    converge_result_kernel<<<1, 64, 0, s>>>(ctl, max_iters, out);
    return hipGetLastError();
}

hipError_t launch_export_centres(const Workspace& ws, const Grid& g, float* out, int32_t* counts,
                                 hipStream_t s) {
    KernelTimer t("export_centres", s);
    export_centres_kernel<<<(g.K + 255) / 256, 256, 0, s>>>(g.K, ws.cen, ws.counts, out, counts);
    return hipGetLastError();
}

hipError_t launch_import_centres(const Workspace& ws, const Grid& g, const float* in,
                                 hipStream_t s) {
    KernelTimer t("import_centres", s);
    import_centres_kernel<<<(g.K + 255) / 256, 256, 0, s>>>(g.K, in, ws.cen);
    return hipGetLastError();
}

}  // namespace slic
