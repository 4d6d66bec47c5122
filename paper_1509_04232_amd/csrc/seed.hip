// Cluster centre initialisation (Section 3: one thread per centre fills the
// superpixel map) with the perturbation of Section 2: the seed moves to the
// lowest-gradient pixel of its 3x3 window.
//
// Seed of cell (cx, cy): the cell's middle pixel x0 + (x1 - x0 - 1) / 2 (and
// likewise in y), where the cell spans [x0, x1) clipped to the image.
// Gradient (that of the SLIC paper the method builds on):
//   G(x, y) = |I(x+1, y) - I(x-1, y)|^2 + |I(x, y+1) - I(x, y-1)|^2
// over the Lab vector, coordinates clamped to the image.  The window is
// scanned row by row and the seed moves only on a strictly smaller G.
// The kernel also clears the centre's count and the first accumulators.
#include "slic_internal.h"

#pragma clang fp contract(off)

namespace slic {
namespace {

__device__ __forceinline__ float norm2(float u, float v, float t) {
    float a = u * u;
    a = a + v * v;
    a = a + t * t;
    return a;
}

__device__ float gradient(const float* __restrict__ L, const float* __restrict__ A,
                          const float* __restrict__ B, int w, int h, int x, int y) {
    const int xl = max(x - 1, 0), xr = min(x + 1, w - 1);
    const int yu = max(y - 1, 0), yd = min(y + 1, h - 1);
    const size_t row = static_cast<size_t>(y) * w;
    const float gx = norm2(L[row + xr] - L[row + xl], A[row + xr] - A[row + xl],
                           B[row + xr] - B[row + xl]);
    const size_t up = static_cast<size_t>(yu) * w + x, dn = static_cast<size_t>(yd) * w + x;
    const float gy = norm2(L[dn] - L[up], A[dn] - A[up], B[dn] - B[up]);
    return gx + gy;
}

// Nine threads per seed, one per window position; the first thread of each
// group then applies the sequential rule (start at the middle pixel, scan the
// window row by row, move only on a strictly smaller gradient).
constexpr int kSeedBlock = 256;
constexpr int kSeedsPerBlock = kSeedBlock / 9;

__global__ __launch_bounds__(kSeedBlock) void seed_kernel(const float* __restrict__ L,
                                                          const float* __restrict__ A,
                                                          const float* __restrict__ B, int w,
                                                          int h, int S, int ns_c, int K,
                                                          int perturb, float* __restrict__ cen,
                                                          int32_t* __restrict__ counts,
                                                          long long* __restrict__ sums) {
    __shared__ float grad[kSeedBlock];
    const int sl = threadIdx.x / 9, pos = threadIdx.x % 9;
    const int k = blockIdx.x * kSeedsPerBlock + sl;
    const bool active = sl < kSeedsPerBlock && k < K;
    int sx = 0, sy = 0;
    if (active) {
        const int cx = k % ns_c, cy = k / ns_c;
        const int x0 = cx * S, x1 = min(x0 + S, w);
        const int y0 = cy * S, y1 = min(y0 + S, h);
        sx = x0 + (x1 - x0 - 1) / 2;
        sy = y0 + (y1 - y0 - 1) / 2;
        const int nx = sx + pos % 3 - 1, ny = sy + pos / 3 - 1;
        float g = __builtin_huge_valf();
        if (perturb && nx >= 0 && nx < w && ny >= 0 && ny < h)
            g = gradient(L, A, B, w, h, nx, ny);
        grad[threadIdx.x] = g;
    }
    __syncthreads();
    if (!active || pos != 0) return;
    int bx = sx, by = sy;
    if (perturb) {
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
    const size_t i = static_cast<size_t>(by) * w + bx;
    float4* c = reinterpret_cast<float4*>(cen + static_cast<size_t>(k) * kCenStride);
    c[0] = make_float4(L[i], A[i], B[i], static_cast<float>(bx));
    c[1] = make_float4(static_cast<float>(by), 0.0f, 0.0f, 0.0f);
    counts[k] = 0;
    long long* s = sums + static_cast<size_t>(k) * kSumStride;
#pragma unroll
    for (int j = 0; j < kSumStride; ++j) s[j] = 0;
}

}  // namespace

hipError_t launch_seed(const Workspace& ws, int32_t w, int32_t h, const Grid& g, int perturb,
                       hipStream_t s) {
    const int grid = (g.K + kSeedsPerBlock - 1) / kSeedsPerBlock;
    KernelTimer t("seed", s);
    seed_kernel<<<grid, kSeedBlock, 0, s>>>(ws.L, ws.A, ws.B, w, h, g.S, g.ns_c, g.K, perturb, ws.cen,
                                       ws.counts, ws.sums);
    return hipGetLastError();
}

}  // namespace slic
