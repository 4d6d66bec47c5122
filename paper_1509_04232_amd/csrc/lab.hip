// Image space conversion (Section 3): sRGB bytes -> planar FP32 CIELAB,
// one thread per pixel.
//
// Definition: sRGB decoding (IEC 61966-2-1) through a 256-entry table, the
// sRGB->XYZ matrix with each row divided by its sum (so the D65 white maps
// to X = Y = Z = 1), the CIE f(t) in FP64 (cube root by Newton's method
// above (6/29)^3, the linear segment below), then L = 116 fy - 16,
// a = 500 (fx - fy), b = 200 (fy - fz) in FP32.  Every operation is IEEE
// round-to-nearest in the order written; the file is compiled without FMA
// contraction.
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

// Cube root of a normal, positive double by Newton's method on y^3 = t.
// The exponent is split off so that the iteration runs on g in [0.5, 4):
// t = f * 2^e, f in [0.5, 1), e = 3q + r with r in {0,1,2}, g = f * 2^r,
// cbrt(t) = cbrt(g) * 2^q.  Quadratic seed, four steps of
// y <- (2 y^3 + g) / (3 y^2).
__device__ __forceinline__ double newton_cbrt(double t) {
    const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(t));
    const int e = static_cast<int>((bits >> 52) & 0x7ffull) - 1022;
    const double f = __longlong_as_double(
        static_cast<long long>((bits & 0x800fffffffffffffull) | 0x3fe0000000000000ull));
    const int r = ((e % 3) + 3) % 3;
    const int q = (e - r) / 3;
    const double g = f * static_cast<double>(1 << r);
    const double lin = 0.6052 + 0.4255 * g;
    const double g2 = g * g;
    double y = lin - 0.04658 * g2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double y2 = y * y;
        const double y3 = y2 * y;
        double num = 2.0 * y3;
        num = num + g;
        const double den = 3.0 * y2;
        y = num / den;
    }
    // 2^q as a double (q is small: t lies in (0.0088, 1.1])
    const double scale =
        __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(q + 1023) << 52));
    return y * scale;
}

__device__ __forceinline__ float cie_f(float t) {
    const double td = static_cast<double>(t);
    const double eps = 216.0 / 24389.0;
    const double kappa = 24389.0 / 27.0;
    double r;
    if (td > eps) {
        r = newton_cbrt(td);
    } else {
        const double p = kappa * td;
        const double s = p + 16.0;
        r = s / 116.0;
    }
    return static_cast<float>(r);
}

constexpr int kLabBlockX = 64, kLabBlockY = 4;

__global__ __launch_bounds__(kLabBlockX* kLabBlockY) void lab_kernel(
    const uint8_t* __restrict__ rgb, int32_t w, int32_t h, int32_t pitch, int32_t channels,
    float* __restrict__ L, float* __restrict__ A, float* __restrict__ B, LabTables tab) {
    __shared__ float lin[256];
    const int tid = threadIdx.y * kLabBlockX + threadIdx.x;
    lin[tid] = tab.lin[tid];
    __syncthreads();
    const int x = blockIdx.x * kLabBlockX + threadIdx.x;
    const int y = blockIdx.y * kLabBlockY + threadIdx.y;
    if (x >= w || y >= h) return;
    const uint8_t* p = rgb + static_cast<size_t>(y) * pitch + static_cast<size_t>(x) * channels;
    const float r = lin[p[0]], g = lin[p[1]], b = lin[p[2]];
    float X = tab.nm[0] * r;
    X = X + tab.nm[1] * g;
    X = X + tab.nm[2] * b;
    float Y = tab.nm[3] * r;
    Y = Y + tab.nm[4] * g;
    Y = Y + tab.nm[5] * b;
    float Z = tab.nm[6] * r;
    Z = Z + tab.nm[7] * g;
    Z = Z + tab.nm[8] * b;
    const float fx = cie_f(X), fy = cie_f(Y), fz = cie_f(Z);
    const size_t i = static_cast<size_t>(y) * w + x;
    const float l = 116.0f * fy;
    L[i] = l - 16.0f;
    const float dxy = fx - fy;
    A[i] = 500.0f * dxy;
    const float dyz = fy - fz;
    B[i] = 200.0f * dyz;
}

}  // namespace

hipError_t launch_lab(const uint8_t* rgb, int32_t w, int32_t h, int32_t pitch, int32_t channels,
                      float* L, float* A, float* B, hipStream_t s) {
    static const LabTables tab = make_tables();
    dim3 block(kLabBlockX, kLabBlockY);
    dim3 grid((w + kLabBlockX - 1) / kLabBlockX, (h + kLabBlockY - 1) / kLabBlockY);
    KernelTimer t("lab", s);
    lab_kernel<<<grid, block, 0, s>>>(rgb, w, h, pitch, channels, L, A, B, tab);
    return hipGetLastError();
}

}  // namespace slic
