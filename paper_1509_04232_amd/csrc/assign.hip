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
// multiply-adds and the hardware square root, keeping the smallest and the
// second smallest value.  Each fast value is within 11 u of the exact real
// distance and each reference value within 4 u (u = 2^-24; relative, all
// terms are non-negative), so if the best fast value is below the second
// smallest by more than 2^-18 of the latter, the reference argmin is the same
// candidate and no reference value can tie with it.  Otherwise (near ties)
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
#include "slic_internal.h"

#pragma clang fp contract(off)

namespace slic {
namespace {

constexpr int kTileX = 32;       // pixels per workgroup row
constexpr int kThreads = 256;    // 32 x 8 threads; each thread owns PPT rows
constexpr float kCertify = 0x1p-18f;

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

// Fast Eq. 1 distance (fused multiply-adds, hardware square root).
__device__ __forceinline__ float eq1_fast(float cl, float ca, float cb, float cx, float cy, float l,
                                          float a, float b, float xf, float yf, float wgt) {
    const float dl = cl - l, da = ca - a, db = cb - b;
    const float s = __builtin_fmaf(db, db, __builtin_fmaf(da, da, dl * dl));
    const float dx = cx - xf, dy = cy - yf;
    const float t = __builtin_fmaf(dy, dy, dx * dx);
    return __builtin_fmaf(wgt, __builtin_amdgcn_sqrtf(t), __builtin_amdgcn_sqrtf(s));
}

struct AssignArgs {
    const float* L;
    const float* A;
    const float* B;
    int w, h, S, ns_c, ns_r;
    float wgt;
    float* cen;            // K x kCenStride: centres used by the last launch
    int32_t* counts;       // K
    int32_t* labels;       // N
    long long* sums_prev;  // read (mean half), or null on the first launch
    long long* sums_acc;   // accumulated by this launch
    long long* sums_next;  // cleared by this launch (owners)
};

// Shared-memory layout (dynamic): for every cell of the staged window
// (the workgroup's cells plus a one-cell ring, out-of-grid cells included):
//   float4 cen4[n] (L, a, b, x), float ceny[n], int kidx[n] (-1: none),
//   u64 bins[4][n] (sum qL, sum qa, sum qb, packed x'|y'<<20|count<<40).
__host__ __device__ inline size_t assign_lds_bytes(int ncells) {
    return static_cast<size_t>(ncells) * (16 + 4 + 4 + 32);
}

template <int PPT>
__global__ __launch_bounds__(kThreads) void assign_kernel(AssignArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kTileY = 8 * PPT;
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
    const int S = g.S;
    const int gx_lo = x0 / S - 1, gy_lo = y0 / S - 1;
    const int gx_hi = (min(x0 + kTileX, g.w) - 1) / S + 1;
    const int gy_hi = (min(y0 + kTileY, g.h) - 1) / S + 1;
    const int ncx = gx_hi - gx_lo + 1, ncy = gy_hi - gy_lo + 1, ncells = ncx * ncy;
    float4* cen4 = reinterpret_cast<float4*>(smem);
    float* ceny = reinterpret_cast<float*>(cen4 + ncells);
    int* kidx = reinterpret_cast<int*>(ceny + ncells);
    unsigned long long* bins = reinterpret_cast<unsigned long long*>(
        reinterpret_cast<uintptr_t>(kidx + ncells + 1) & ~static_cast<uintptr_t>(7));

    // ---- stage the candidate centres (and, from the second launch on,
    // derive them from the previous launch's sums)
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
        const bool owner = (cx * S) / kTileX == static_cast<int>(blockIdx.x) &&
                           (cy * S) / kTileY == static_cast<int>(blockIdx.y);
        float* c = g.cen + static_cast<size_t>(k) * kCenStride;
        float4 v;
        float vy;
        if (g.sums_prev) {
            const long long* s = g.sums_prev + static_cast<size_t>(k) * kSumStride;
            const long long n = s[5];
            if (n > 0) {
                const double dn = static_cast<double>(n);
                const double inv = 1.0 / static_cast<double>(1 << kQShift);
                const double ml = static_cast<double>(s[0]) / dn;
                const double ma = static_cast<double>(s[1]) / dn;
                const double mb = static_cast<double>(s[2]) / dn;
                v = make_float4(static_cast<float>(ml * inv), static_cast<float>(ma * inv),
                                static_cast<float>(mb * inv),
                                static_cast<float>(static_cast<double>(s[3]) / dn));
                vy = static_cast<float>(static_cast<double>(s[4]) / dn);
                if (owner) {
                    *reinterpret_cast<float4*>(c) = v;
                    c[4] = vy;
                }
            } else {
                v = *reinterpret_cast<const float4*>(c);
                vy = c[4];
            }
            if (owner) g.counts[k] = static_cast<int32_t>(n);
        } else {
            v = *reinterpret_cast<const float4*>(c);
            vy = c[4];
        }
        if (owner) {
            long long* z = g.sums_next + static_cast<size_t>(k) * kSumStride;
            for (int j = 0; j < kSumStride; ++j) z[j] = 0;
        }
        cen4[i] = v;
        ceny[i] = vy;
    }
    __syncthreads();

    // ---- associate PPT vertically adjacent pixels per thread
    const int tx = threadIdx.x % kTileX, ty = threadIdx.x / kTileX;
    const int x = x0 + tx;
    const float xf = static_cast<float>(x);
    const int gx_rel = (x < g.w ? x / S : 0) - gx_lo - 1;  // window column of the left candidate
    const float scale = static_cast<float>(1 << kQShift);
    int run_cell = -1;
    int rl = 0, ra = 0, rb = 0;
    unsigned long long rxyc = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int y = y0 + ty * PPT + j;
        const bool valid = x < g.w && y < g.h;
        if (!valid) continue;
        const size_t pi = static_cast<size_t>(y) * g.w + x;
        const float l = g.L[pi], a = g.A[pi], b = g.B[pi];
        const float yf = static_cast<float>(y);
        const int base = (y / S - gy_lo - 1) * ncx + gx_rel;
        float best = __builtin_huge_valf(), second = __builtin_huge_valf();
        int slot = 0;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const int li = base + (c / 3) * ncx + (c % 3);
            const float4 q = cen4[li];
            const float d = eq1_fast(q.x, q.y, q.z, q.w, ceny[li], l, a, b, xf, yf, g.wgt);
            second = fminf(second, fmaxf(best, d));
            slot = d < best ? c : slot;
            best = fminf(best, d);
        }
        if (!(best < __builtin_fmaf(second, -kCertify, second))) {
            // near tie: reference values, lowest index wins ties
            float bref = __builtin_huge_valf();
            slot = -1;
            for (int c = 0; c < 9; ++c) {
                const int li = base + (c / 3) * ncx + (c % 3);
                const float4 q = cen4[li];
                const float d = eq1_reference(q.x, q.y, q.z, q.w, ceny[li], l, a, b, xf, yf, g.wgt);
                if (slot < 0 || d < bref) {
                    bref = d;
                    slot = c;
                }
            }
        }
        const int cell = base + (slot / 3) * ncx + (slot % 3);
        g.labels[pi] = kidx[cell];
        const int ql = static_cast<int>(rintf(l * scale));
        const int qa = static_cast<int>(rintf(a * scale));
        const int qb = static_cast<int>(rintf(b * scale));
        const unsigned long long xyc = static_cast<unsigned long long>(x - x0) |
                                       (static_cast<unsigned long long>(y - y0) << 20) |
                                       (1ull << 40);
        if (cell != run_cell) {
            if (run_cell >= 0) {
                atomicAdd(bins + run_cell, static_cast<unsigned long long>(static_cast<long long>(rl)));
                atomicAdd(bins + ncells + run_cell,
                          static_cast<unsigned long long>(static_cast<long long>(ra)));
                atomicAdd(bins + 2 * ncells + run_cell,
                          static_cast<unsigned long long>(static_cast<long long>(rb)));
                atomicAdd(bins + 3 * ncells + run_cell, rxyc);
            }
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
    if (run_cell >= 0) {
        atomicAdd(bins + run_cell, static_cast<unsigned long long>(static_cast<long long>(rl)));
        atomicAdd(bins + ncells + run_cell, static_cast<unsigned long long>(static_cast<long long>(ra)));
        atomicAdd(bins + 2 * ncells + run_cell,
                  static_cast<unsigned long long>(static_cast<long long>(rb)));
        atomicAdd(bins + 3 * ncells + run_cell, rxyc);
    }
    __syncthreads();

    // ---- add the workgroup's bins to the global sums
    for (int i = threadIdx.x; i < ncells; i += kThreads) {
        const unsigned long long p = bins[3 * ncells + i];
        const long long n = static_cast<long long>(p >> 40);
        if (n == 0) continue;
        const long long sx = static_cast<long long>(p & 0xFFFFFull) + n * x0;
        const long long sy = static_cast<long long>((p >> 20) & 0xFFFFFull) + n * y0;
        unsigned long long* s =
            reinterpret_cast<unsigned long long*>(g.sums_acc + static_cast<size_t>(kidx[i]) * kSumStride);
        atomicAdd(s + 0, bins[i]);
        atomicAdd(s + 1, bins[ncells + i]);
        atomicAdd(s + 2, bins[2 * ncells + i]);
        atomicAdd(s + 3, static_cast<unsigned long long>(sx));
        atomicAdd(s + 4, static_cast<unsigned long long>(sy));
        atomicAdd(s + 5, static_cast<unsigned long long>(n));
    }
}

constexpr int kEnergyBlock = 256;

__global__ __launch_bounds__(kEnergyBlock) void energy_kernel(
    const float* __restrict__ L, const float* __restrict__ A, const float* __restrict__ B, int w,
    int n, float wgt, const float* __restrict__ cen, const int32_t* __restrict__ labels,
    double* __restrict__ partial) {
    __shared__ double red[kEnergyBlock];
    const int i = blockIdx.x * kEnergyBlock + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const float* c = cen + static_cast<size_t>(labels[i]) * kCenStride;
        v = static_cast<double>(eq1_reference(c[0], c[1], c[2], c[3], c[4], L[i], A[i], B[i],
                                              static_cast<float>(i % w),
                                              static_cast<float>(i / w), wgt));
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

template <int PPT>
hipError_t launch_assign_ppt(const AssignArgs& a, hipStream_t s) {
    constexpr int kTileY = 8 * PPT;
    dim3 grid((a.w + kTileX - 1) / kTileX, (a.h + kTileY - 1) / kTileY);
    // window of cells over any tile: at most (tile/S + 3) per side
    const int ncx = (kTileX - 1) / a.S + 3 + 1, ncy = (kTileY - 1) / a.S + 3 + 1;
    const size_t lds = assign_lds_bytes(ncx * ncy) + 16;
    KernelTimer t("assign", s);
    assign_kernel<PPT><<<grid, kThreads, lds, s>>>(a);
    return hipGetLastError();
}

}  // namespace

int assign_pixels_per_thread(int32_t w, int32_t h) {
    // enough workgroups to fill 256 compute units several times over
    const long long n = static_cast<long long>(w) * h;
    if (n >= (4ll << 20)) return 4;
    if (n >= (1ll << 20)) return 2;
    return 1;
}

hipError_t launch_assign(const Workspace& ws, int32_t w, int32_t h, const Grid& g, int64_t t,
                         int ppt, hipStream_t s) {
    AssignArgs a;
    a.L = ws.L;
    a.A = ws.A;
    a.B = ws.B;
    a.w = w;
    a.h = h;
    a.S = g.S;
    a.ns_c = g.ns_c;
    a.ns_r = g.ns_r;
    a.wgt = g.w;
    a.cen = ws.cen;
    a.counts = ws.counts;
    a.labels = ws.labels;
    const size_t stride = static_cast<size_t>(g.K) * kSumStride;
    a.sums_acc = ws.sums + stride * static_cast<size_t>(t % 3);
    a.sums_prev = t > 0 ? ws.sums + stride * static_cast<size_t>((t + 2) % 3) : nullptr;
    a.sums_next = ws.sums + stride * static_cast<size_t>((t + 1) % 3);
    if (ppt <= 0) ppt = assign_pixels_per_thread(w, h);
    // keep the staged window within 64 KiB of LDS
    while (ppt > 1 && assign_lds_bytes(((kTileX - 1) / g.S + 4) * ((8 * ppt - 1) / g.S + 4)) + 16 >
                          (64u << 10))
        ppt /= 2;
    switch (ppt) {
        case 1: return launch_assign_ppt<1>(a, s);
        case 2: return launch_assign_ppt<2>(a, s);
        case 4: return launch_assign_ppt<4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_energy(const Workspace& ws, int32_t w, int32_t h, const Grid& g, double* out,
                         hipStream_t s) {
    const int n = w * h;
    const int nb = (n + kEnergyBlock - 1) / kEnergyBlock;
    {
        KernelTimer t("energy", s);
        energy_kernel<<<nb, kEnergyBlock, 0, s>>>(ws.L, ws.A, ws.B, w, n, g.w, ws.cen, ws.labels,
                                                  ws.partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    KernelTimer t("energy_final", s);
    energy_final_kernel<<<1, kEnergyBlock, 0, s>>>(ws.partial, nb, static_cast<double>(n), out);
    return hipGetLastError();
}

hipError_t launch_export_centres(const Workspace& ws, const Grid& g, float* out, int32_t* counts,
                                 hipStream_t s) {
    KernelTimer t("export_centres", s);
    export_centres_kernel<<<(g.K + 255) / 256, 256, 0, s>>>(g.K, ws.cen, ws.counts, out, counts);
    return hipGetLastError();
}

}  // namespace slic
