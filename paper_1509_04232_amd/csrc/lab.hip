// Image space conversion (Section 3: sRGB bytes -> planar FP32 CIELAB, one
// thread per pixel) fused with cluster centre initialisation (Section 3: the
// superpixel map) and the seed perturbation of Section 2.
//
// Conversion: sRGB decoding (IEC 61966-2-1) through a 256-entry table, the
// sRGB->XYZ matrix with each row divided by its sum (so the D65 white maps
// to X = Y = Z = 1), the CIE f(t) in FP64 (cube root above (6/29)^3, the
// linear segment below), then L = 116 fy - 16, a = 500 (fx - fy),
// b = 200 (fy - fz) in FP32.  Every operation is IEEE round-to-nearest in
// the order written; the file is compiled without FMA contraction (the cube
// root's fused multiply-adds are explicit).  The cube root's result is that
// of Newton's method as written below (newton_cbrt), rounded to FP32, reached
// by a certified cheaper estimate wherever that provably rounds the same.  The colour-space option yields
// XYZ scaled by 100 (same order, then the scaling) or the R, G, B bytes as
// floats instead; the seeds and the gradient work on whichever planes.
//
// Seeds: the seed of cell (cx, cy) is the cell's middle pixel
// x0 + (x1 - x0 - 1) / 2 (likewise in y), the cell spanning [x0, x1)
// clipped to the image.  With perturbation it moves to the pixel of its 3x3
// window with the smallest gradient (that of the SLIC paper the method builds
// on), G = |I(x+1,y) - I(x-1,y)|^2 + |I(x,y+1) - I(x,y-1)|^2 over the Lab
// vector with coordinates clamped to the image; the window is scanned row by
// row and the seed moves only on a strictly smaller G.  The centre takes the
// chosen pixel's Lab and position; its count and first accumulators are
// cleared.
//
// Each workgroup converts a tile plus a two-pixel halo into LDS, stores the
// tile, and seeds every cell whose middle pixel lies in the tile: the window
// and the gradient's neighbours stay within two pixels of that pixel.
#include <atomic>
#include <cmath>

#include "slic_internal.h"

#pragma clang fp contract(off)

namespace slic {
namespace {

struct LabTables {
    float lin[256];
    float nm[9];
};

// Built on the host in FP64 and rounded once to FP32.
LabTables make_tables() {
    LabTables t;
    for (int v = 0; v < 256; ++v) {
        const double c = static_cast<double>(v) / 255.0;
        const double d = c <= 0.04045 ? c / 12.92 : std::pow((c + 0.055) / 1.055, 2.4);
        t.lin[v] = static_cast<float>(d);
    }
    const double srgb_to_xyz[9] = {0.4124, 0.3576, 0.1805, 0.2126, 0.7152,
                                   0.0722, 0.0193, 0.1192, 0.9505};
    for (int row = 0; row < 3; ++row) {
        const double* m = srgb_to_xyz + 3 * row;
        const double white = (m[0] + m[1]) + m[2];
        for (int col = 0; col < 3; ++col) t.nm[3 * row + col] = static_cast<float>(m[col] / white);
    }
    return t;
}

// Cube root of a normal, positive double.  The exponent is split off so the
// iteration runs on g in [0.5, 4): t = f * 2^e, f in [0.5, 1), e = 3q + r
// with r in {0,1,2}, g = f * 2^r, cbrt(t) = cbrt(g) * 2^q.  Newton's method
// on the inverse cube root (no division): quadratic seed, four steps of
// y <- y + y (1 - g y^3) / 3, then cbrt(g) = g * y * y.
__device__ __forceinline__ double newton_cbrt(double t) {
    const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(t));
    const int e = static_cast<int>((bits >> 52) & 0x7ffull) - 1022;
    const double f = __longlong_as_double(
        static_cast<long long>((bits & 0x800fffffffffffffull) | 0x3fe0000000000000ull));
    const int r = ((e % 3) + 3) % 3;
    const int q = (e - r) / 3;
    const double g = f * static_cast<double>(1 << r);
    const double lin = 1.405 - 0.4258 * g;
    const double g2 = g * g;
    double y = lin + 0.05965 * g2;
    const double third = 1.0 / 3.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double y2 = y * y;
        const double y3 = y2 * y;
        const double err = __builtin_fma(-g, y3, 1.0);
        const double corr = y * err;
        y = __builtin_fma(corr, third, y);
    }
    double c = g * y;
    c = c * y;
    // 2^q as a double (q is small: t lies in (0.0088, 1.1])
    const double scale =
        __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(q + 1023) << 52));
    return c * scale;
}

// The float that newton_cbrt(t) rounds to, for t in (216/24389, 1.1]: a
// cheaper estimate c of the cube root (the inverse cube root seeded by the
// hardware base-2 logarithm and exponential in FP32, then two Newton steps
// in FP64; both c and newton_cbrt lie within about 2^-49 of the exact root)
// is kept where it lies farther than 2^-40 (relative) from both midpoints
// between its FP32 rounding and the neighbouring floats, since newton_cbrt
// then rounds to the same float; elsewhere (about one value in 2^15)
// newton_cbrt runs.
__device__ __forceinline__ float cbrt_rounded(double td) {
    const float tf = static_cast<float>(td);
    const float z0 = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(tf) * (-1.0f / 3.0f));
    double z = static_cast<double>(z0);
    const double third = 1.0 / 3.0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double z2 = z * z;
        const double z3 = z2 * z;
        const double err = __builtin_fma(-td, z3, 1.0);
        const double corr = z * err;
        z = __builtin_fma(corr, third, z);
    }
    double c = td * z;
    c = c * z;
    const float cf = static_cast<float>(c);
    const double fc = static_cast<double>(cf);
    const double up = static_cast<double>(__int_as_float(__float_as_int(cf) + 1));
    const double dn = static_cast<double>(__int_as_float(__float_as_int(cf) - 1));
    const double margin = c * 0x1p-40;
    if (c < 0.5 * (fc + up) - margin && c > 0.5 * (fc + dn) + margin) return cf;
    return static_cast<float>(newton_cbrt(td));
}

__device__ __forceinline__ float cie_f(float t) {
    const double td = static_cast<double>(t);
    const double eps = 216.0 / 24389.0;
    const double kappa = 24389.0 / 27.0;
    if (td > eps) return cbrt_rounded(td);
    const double p = kappa * td;
    const double s = p + 16.0;
    return static_cast<float>(s / 116.0);
}

__device__ __forceinline__ void rgb_to_lab(const float* lin, const float* nm, const uint8_t* p,
                                           float* L, float* A, float* B) {
    const float r = lin[p[0]], g = lin[p[1]], b = lin[p[2]];
    float X = nm[0] * r;
    X = X + nm[1] * g;
    X = X + nm[2] * b;
    float Y = nm[3] * r;
    Y = Y + nm[4] * g;
    Y = Y + nm[5] * b;
    float Z = nm[6] * r;
    Z = Z + nm[7] * g;
    Z = Z + nm[8] * b;
    const float fx = cie_f(X), fy = cie_f(Y), fz = cie_f(Z);
    const float l = 116.0f * fy;
    *L = l - 16.0f;
    const float dxy = fx - fy;
    *A = 500.0f * dxy;
    const float dyz = fy - fz;
    *B = 200.0f * dyz;
}

// XYZ scaled by 100 (the colour-space option), in the Lab path's order.
__device__ __forceinline__ void rgb_to_xyz100(const float* lin, const float* nm, const uint8_t* p,
                                              float* X0, float* Y0, float* Z0) {
    const float r = lin[p[0]], g = lin[p[1]], b = lin[p[2]];
    float X = nm[0] * r;
    X = X + nm[1] * g;
    X = X + nm[2] * b;
    float Y = nm[3] * r;
    Y = Y + nm[4] * g;
    Y = Y + nm[5] * b;
    float Z = nm[6] * r;
    Z = Z + nm[7] * g;
    Z = Z + nm[8] * b;
    *X0 = 100.0f * X;
    *Y0 = 100.0f * Y;
    *Z0 = 100.0f * Z;
}

__device__ __forceinline__ float norm2(float u, float v, float t) {
    float a = u * u;
    a = a + v * v;
    a = a + t * t;
    return a;
}

constexpr int kTW = 64, kTH = 32, kHalo = 2;  // the tile of batches and large frames
constexpr int kThreads = 1024;
// Smaller frames: the kernel is bound by its cube roots, so the time is set
// by the conversions (tile plus halo) of the busiest compute unit.  With
// 64 x 32 tiles a 320 x 240 frame keeps 40 units busy and a 640 x 480 frame
// 150; the smallest tile whose count still fits one workgroup per unit
// spreads the work: 32 x 16 (720 conversions each) or 40 x 30 (1,496; 256
// tiles at 640 x 480), else 64 x 32 (2,448), whose halo costs least when
// every unit gets several tiles.  (32 x 16 tiles at 640 x 480, three per
// unit, were slower than 64 x 32.)
constexpr int kSmallTW = 32, kSmallTH = 16, kSmallThreads = 512;
constexpr int kMidTW = 40, kMidTH = 30;

// kBatch: the workgroup's image comes from the tile map (a batch) rather
// than the kernel argument; separate instantiations, so a single-image
// launch reads no table and takes no branch on the way in.  TW x TH: the
// tile (plus a kHalo ring), NT threads.
template <bool kBatch, int TW, int TH, int NT>
__global__ __launch_bounds__(NT) void lab_seed_kernel(LabSeedImage single, LabSeedTileMap map,
                                                      LabTables tab) {
    constexpr int kSW = TW + 2 * kHalo, kSH = TH + 2 * kHalo;  // staged tile
    constexpr int kSeedsPerPass = NT / 9;
    static_assert(NT >= 256, "the sRGB table is loaded by the first 256 threads");
    __shared__ float lin[256];
    __shared__ float sL[kSW * kSH], sA[kSW * kSH], sB[kSW * kSH];
    __shared__ float grad[NT];
    if (threadIdx.x < 256) lin[threadIdx.x] = tab.lin[threadIdx.x];
    LabSeedImage g;
    int bx, by;
    if constexpr (kBatch) {  // batch: this workgroup's image from the tile map
        const int img = map.tile_image[blockIdx.x];
        g = map.images[img];
        const int local = static_cast<int>(blockIdx.x) - map.tile_first[img];
        bx = local % g.tiles_x;
        by = local / g.tiles_x;
    } else {
        g = single;
        bx = blockIdx.x;
        by = blockIdx.y;
    }
    __syncthreads();
    const int x0 = bx * TW, y0 = by * TH;

    // ---- convert the tile and its halo
    for (int i = threadIdx.x; i < kSW * kSH; i += NT) {
        const int x = x0 - kHalo + i % kSW, y = y0 - kHalo + i / kSW;
        if (x < 0 || y < 0 || x >= g.w || y >= g.h) continue;
        float l, a, b;
        const uint8_t* px = g.rgb + static_cast<size_t>(y) * g.pitch + static_cast<size_t>(x) * g.channels;
        if (g.space == 0) {
            rgb_to_lab(lin, tab.nm, px, &l, &a, &b);
        } else if (g.space == 1) {
            rgb_to_xyz100(lin, tab.nm, px, &l, &a, &b);
        } else {
            l = static_cast<float>(px[0]);
            a = static_cast<float>(px[1]);
            b = static_cast<float>(px[2]);
        }
        sL[i] = l;
        sA[i] = a;
        sB[i] = b;
        if (x >= x0 && x < x0 + TW && y >= y0 && y < y0 + TH) {
            const size_t pi = static_cast<size_t>(y) * g.w + x;
            g.L[pi] = l;
            g.A[pi] = a;
            g.B[pi] = b;
        }
    }
    __syncthreads();

    // ---- cells whose middle pixel lies in this tile
    const int S = g.S;
    auto middle = [&](int c, int extent) {
        const int lo = c * S, hi = min(lo + S, extent);
        return lo + (hi - lo - 1) / 2;
    };
    int cx0 = x0 / S, cx1 = min((x0 + TW - 1) / S, g.ns_c - 1);
    if (middle(cx0, g.w) < x0) ++cx0;
    if (cx1 >= cx0 && middle(cx1, g.w) >= x0 + TW) --cx1;
    int cy0 = y0 / S, cy1 = min((y0 + TH - 1) / S, g.ns_r - 1);
    if (middle(cy0, g.h) < y0) ++cy0;
    if (cy1 >= cy0 && middle(cy1, g.h) >= y0 + TH) --cy1;
    const int ncx = cx1 - cx0 + 1, ncy = cy1 - cy0 + 1;
    if (ncx <= 0 || ncy <= 0) return;  // uniform across the workgroup
    const int nseeds = ncx * ncy;
    auto at = [&](int x, int y) { return (y - y0 + kHalo) * kSW + (x - x0 + kHalo); };
    for (int base = 0; base < nseeds; base += kSeedsPerPass) {
        const int sl = threadIdx.x / 9, pos = threadIdx.x % 9;
        const int s = base + sl;
        const bool active = sl < kSeedsPerPass && s < nseeds;
        int cx = 0, cy = 0, sx = 0, sy = 0;
        if (active) {
            cx = cx0 + s % ncx;
            cy = cy0 + s / ncx;
            sx = middle(cx, g.w);
            sy = middle(cy, g.h);
            const int nx = sx + pos % 3 - 1, ny = sy + pos / 3 - 1;
            float gv = __builtin_huge_valf();
            if (g.perturb && nx >= 0 && nx < g.w && ny >= 0 && ny < g.h) {
                const int xl = max(nx - 1, 0), xr = min(nx + 1, g.w - 1);
                const int yu = max(ny - 1, 0), yd = min(ny + 1, g.h - 1);
                const int il = at(xl, ny), ir = at(xr, ny), iu = at(nx, yu), id = at(nx, yd);
                const float gx = norm2(sL[ir] - sL[il], sA[ir] - sA[il], sB[ir] - sB[il]);
                const float gy = norm2(sL[id] - sL[iu], sA[id] - sA[iu], sB[id] - sB[iu]);
                gv = gx + gy;
            }
            grad[threadIdx.x] = gv;
        }
        __syncthreads();
        if (active && pos == 0) {
            int bx = sx, by = sy;
            if (g.perturb) {
                const float* gw = grad + threadIdx.x;
                float best = gw[4];  // the middle pixel
                for (int p = 0; p < 9; ++p) {
                    if (gw[p] < best) {  // positions outside the image hold +inf
                        best = gw[p];
                        bx = sx + p % 3 - 1;
                        by = sy + p / 3 - 1;
                    }
                }
            }
            const int k = cy * g.ns_c + cx;
            const int i = at(bx, by);
            float4* c = reinterpret_cast<float4*>(g.cen + static_cast<size_t>(k) * kCenStride);
            c[0] = make_float4(sL[i], sA[i], sB[i], static_cast<float>(bx));
            c[1] = make_float4(static_cast<float>(by), 0.0f, 0.0f, 0.0f);
            g.counts[k] = 0;
            long long* z = g.sums + static_cast<size_t>(k) * kSumStride;
#pragma unroll
            for (int j = 0; j < kSumStride; ++j) z[j] = 0;
        }
        __syncthreads();
    }
}

const LabTables& tables() {
    static const LabTables tab = make_tables();
    return tab;
}

}  // namespace

int lab_seed_tile_w() { return kTW; }
int lab_seed_tile_h() { return kTH; }

LabSeedImage lab_seed_image(const uint8_t* rgb, int32_t w, int32_t h, int32_t pitch,
                            int32_t channels, const Workspace& ws, const Grid& grid, int perturb) {
    LabSeedImage a;
    a.rgb = rgb;
    a.w = w;
    a.h = h;
    a.pitch = pitch;
    a.channels = channels;
    a.L = ws.L;
    a.A = ws.A;
    a.B = ws.B;
    a.S = grid.S;
    a.ns_c = grid.ns_c;
    a.ns_r = grid.ns_r;
    a.perturb = perturb;
    a.space = grid.space;
    a.cen = ws.cen;
    a.counts = ws.counts;
    a.sums = ws.sums;
    a.tiles_x = (w + kTW - 1) / kTW;
    return a;
}

// Compute units of the current device (looked up once per device).
int compute_units() {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int c = cached[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
        c = 256;
    cached[dev].store(c, std::memory_order_relaxed);
    return c;
}

hipError_t launch_lab_seed(const uint8_t* rgb, int32_t w, int32_t h, int32_t pitch,
                           int32_t channels, const Workspace& ws, const Grid& grid, int perturb,
                           hipStream_t s) {
    const LabSeedImage a = lab_seed_image(rgb, w, h, pitch, channels, ws, grid, perturb);
    const LabSeedTileMap none{nullptr, nullptr, nullptr};
    KernelTimer t("lab_seed", s);
    const int cus = compute_units();
    auto tiles = [&](int tw, int th) { return ((w + tw - 1) / tw) * ((h + th - 1) / th); };
    if (tiles(kSmallTW, kSmallTH) <= cus) {
        dim3 g((w + kSmallTW - 1) / kSmallTW, (h + kSmallTH - 1) / kSmallTH);
        lab_seed_kernel<false, kSmallTW, kSmallTH, kSmallThreads>
            <<<g, kSmallThreads, 0, s>>>(a, none, tables());
    } else if (tiles(kMidTW, kMidTH) <= cus) {
        dim3 g((w + kMidTW - 1) / kMidTW, (h + kMidTH - 1) / kMidTH);
        lab_seed_kernel<false, kMidTW, kMidTH, kThreads><<<g, kThreads, 0, s>>>(a, none, tables());
    } else {
        dim3 g((w + kTW - 1) / kTW, (h + kTH - 1) / kTH);
        lab_seed_kernel<false, kTW, kTH, kThreads><<<g, kThreads, 0, s>>>(a, none, tables());
    }
    return hipGetLastError();
}

hipError_t launch_lab_seed_batch(const LabSeedTileMap& map, int total_tiles, hipStream_t s) {
    if (!map.images) return hipErrorInvalidValue;
    LabSeedImage unused{};
    KernelTimer t("lab_seed", s);
    lab_seed_kernel<true, kTW, kTH, kThreads><<<total_tiles, kThreads, 0, s>>>(unused, map, tables());
    return hipGetLastError();
}

}  // namespace slic
