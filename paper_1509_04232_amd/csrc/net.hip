// The learned warm start: a 3x3 convolutional net (3 -> 32 -> 32 -> 9, ReLU
// after the first two layers) that predicts, per pixel, which of the nine
// grid cells around the pixel's own cell holds the centre the pixel ends up
// with after plain SLIC, plus a learned per-phase bias P[(y mod S) S +
// (x mod S)][9] on the logits (the convolutions alone cannot see where in
// its cell a pixel lies).  Activations and convolution weights are bfloat16
// (round to nearest even), accumulation FP32; every convolution runs on MFMA
// (v_mfma_f32_16x16x32_bf16).
//
// Layouts.  Activations are NHWC over a batch of equally sized crops,
// element ((n H + y) W + x) C + c, with C = 32 bf16 channels for the input
// (3 used: L/100, a/128, b/128), both hidden layers and the gradients, and
// C = 16 FP32 for the logits (9 used).  Zero padding at every crop border.
// Parameters are one FP32 vector: W1[9][32][3], b1[32], W2[9][32][32], b2[32],
// W3[9][9][32], b3[9], P[S*S][9], with tap = (dy + 1) * 3 + (dx + 1) reading
// the input at (x + dx, y + dy).
//
// MFMA operands (v_mfma_f32_16x16x32_bf16, D = A B + C with A 16x32 and B
// 32x16): lane l supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16]
// for j = 0..7 and holds D[4 (l / 16) + i][l % 16], i = 0..3.  The forward and
// data-gradient convolutions take A = weights (out x in) and B = activations
// (in x pixels); the weight gradients take A = output gradients (out x
// pixels) and B = inputs (pixels x in).
//
// Training reductions are deterministic: each workgroup writes its partial
// gradient, and one kernel sums the partials in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "slic_internal.h"

namespace slic {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 32;   // hidden (and padded input) channels
constexpr int kC3 = 9;   // classes
constexpr int kOffW1 = 0, kOffB1 = 9 * kC * 3, kOffW2 = kOffB1 + kC;
constexpr int kOffB2 = kOffW2 + 9 * kC * kC, kOffW3 = kOffB2 + kC;
constexpr int kOffB3 = kOffW3 + 9 * kC3 * kC, kOffP = kOffB3 + kC3;
constexpr int kMaxS = 32;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// FP32 -> bf16, round to nearest even (gfx950's v_cvt_pk_bf16_f32).
__device__ __forceinline__ unsigned short bf16_bits(float f) {
    return __builtin_bit_cast(unsigned short, static_cast<__bf16>(f));
}
__device__ __forceinline__ float bf16_float(unsigned short h) {
    return __uint_as_float(static_cast<unsigned>(h) << 16);
}
__device__ __forceinline__ unsigned pack2(float lo, float hi) {
    const bf16x2 v = {static_cast<__bf16>(lo), static_cast<__bf16>(hi)};
    return __builtin_bit_cast(unsigned, v);
}
// The 32 bits starting 16 bits into the 64-bit value hi:lo.
__device__ __forceinline__ unsigned mid16(unsigned hi, unsigned lo) {
    return (lo >> 16) | (hi << 16);
}

struct NetCrop {
    const float* L;
    const float* A;
    const float* B;
    const int32_t* labels;
    int img_w, img_h, ox, oy;
};
constexpr int kMaxCrops = 32;
struct CropTable {
    NetCrop c[kMaxCrops];
};

// bf16 weights in MFMA order: W1b[9][32][32] (inputs 3..31 zero),
// W2b[9][32][32], W3b[9][16][32] (outputs 9..15 zero), and for the data
// gradients the tap-flipped transposes W3t[t][c][o] = W3[8 - t][o][c]
// (o = 9..31 zero) and W2t[t][c][o] = W2[8 - t][o][c].
struct NetWeights {
    unsigned short *W1b, *W2b, *W3b, *W2t, *W3t;
};

// ------------------------------------------------------------- weights

__global__ void prepare_kernel(const float* __restrict__ p, NetWeights wt, int count,
                               float* __restrict__ copy, float* conf_out, float conf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (copy && i < count) copy[i] = p[i];
    if (conf_out && i == 0) *conf_out = conf;
    if (i >= 9 * kC * kC) return;
    const int t = i / (kC * kC), o = (i / kC) % kC, c = i % kC;
    wt.W1b[i] = c < 3 ? bf16_bits(p[kOffW1 + (t * kC + o) * 3 + c]) : 0;
    wt.W2b[i] = bf16_bits(p[kOffW2 + i]);
    // here o indexes the gradient's output (a forward input channel) and c
    // its input (a forward output channel)
    wt.W2t[i] = bf16_bits(p[kOffW2 + ((8 - t) * kC + c) * kC + o]);
    wt.W3t[i] = c < kC3 ? bf16_bits(p[kOffW3 + ((8 - t) * kC3 + c) * kC + o]) : 0;
    if (i < 9 * 16 * kC) {
        const int t3 = i / (16 * kC), o3 = (i / kC) % 16, c3 = i % kC;
        wt.W3b[i] = o3 < kC3 ? bf16_bits(p[kOffW3 + (t3 * kC3 + o3) * kC + c3]) : 0;
    }
}

// --------------------------------------------------------------- input

__global__ __launch_bounds__(256) void input_kernel(CropTable ct, int cw, int ch,
                                                    unsigned short* __restrict__ x) {
    const int per = cw * ch;
    const int px = blockIdx.x * 256 + threadIdx.x;
    const int n = blockIdx.y;
    if (px >= per) return;
    const NetCrop& c = ct.c[n];
    const int gx = c.ox + px % cw, gy = c.oy + px / cw;
    u32x4 v0 = {0u, 0u, 0u, 0u};
    if (gx < c.img_w && gy < c.img_h) {
        const size_t gi = static_cast<size_t>(gy) * c.img_w + gx;
        v0.x = pack2(c.L[gi] / 100.0f, c.A[gi] / 128.0f);
        v0.y = pack2(c.B[gi] / 128.0f, 0.0f);
    }
    u32x4* out = reinterpret_cast<u32x4*>(x + (static_cast<size_t>(n) * per + px) * kC);
    const u32x4 z = {0u, 0u, 0u, 0u};
    out[0] = v0;
    out[1] = z;
    out[2] = z;
    out[3] = z;
}

// ------------------------------------------------- MFMA 3x3 convolution
// 32 bf16 input channels.  A workgroup of four wavefronts covers kTW x 4
// output pixels of one crop, one row per wavefront in N-tiles of 16 pixels;
// the input tile and its one-pixel halo sit in LDS (pixel stride padded to
// 40 elements).  MT tiles of 16 output channels.
enum ConvMode { kFwdRelu = 0, kFwdLogits = 1, kBwdMasked = 2 };

constexpr int kTW = 64, kTRows = 4;
constexpr int kSW = kTW + 2, kSRows = kTRows + 2, kPS = 40;

template <int MT, int MODE>
__global__ __launch_bounds__(256) void conv_kernel(
    const unsigned short* __restrict__ in, const unsigned short* __restrict__ Wb,
    const float* __restrict__ bias, const float* __restrict__ P, CropTable ct, int S, int cw,
    int ch, const unsigned short* __restrict__ mask, unsigned short* __restrict__ out16,
    float* __restrict__ out32) {
    __shared__ __align__(16) unsigned short tile[kSRows * kSW * kPS];
    const int n = blockIdx.z;
    const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTRows;
    const size_t base = static_cast<size_t>(n) * cw * ch;
    for (int i = threadIdx.x; i < kSRows * kSW * 4; i += 256) {
        const int q = i / 4, part = i % 4;
        const int sx = x0 - 1 + q % kSW, sy = y0 - 1 + q / kSW;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (sx >= 0 && sy >= 0 && sx < cw && sy < ch)
            v = reinterpret_cast<const u32x4*>(in + (base + static_cast<size_t>(sy) * cw + sx) * kC)[part];
        *reinterpret_cast<u32x4*>(tile + q * kPS + part * 8) = v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    bf16x8 wa[9][MT];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int m = 0; m < MT; ++m)
            wa[t][m] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const u32x4*>(Wb + ((t * MT * 16 + m * 16 + row) * kC + kq * 8)));
    __syncthreads();
    const int y = y0 + wave;
    if (y >= ch) return;
    for (int nt = 0; nt < kTW / 16; ++nt) {
        const int xs = x0 + nt * 16;
        if (xs >= cw) break;
        f32x4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            // staged position of input pixel (xs + row + dx, y + dy)
            const int q = (wave + t / 3) * kSW + nt * 16 + row + t % 3;
            const bf16x8 b =
                __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(tile + q * kPS + kq * 8));
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][m], b, acc[m], 0, 0, 0);
        }
        // lane holds output channels 16 m + 4 kq + i of pixel xs + row
        const int x = xs + row;
        if (x >= cw) continue;
        const size_t pi = base + static_cast<size_t>(y) * cw + x;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int o0 = m * 16 + kq * 4;
            if constexpr (MODE == kFwdLogits) {
                const NetCrop& c = ct.c[n];
                const int ph = ((c.oy + y) % S) * S + (c.ox + x) % S;
                f32x4 v;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int o = o0 + i;
                    v[i] = o < kC3 ? acc[m][i] + bias[o] + P[ph * kC3 + o] : 0.0f;
                }
                *reinterpret_cast<f32x4*>(out32 + pi * 16 + o0) = v;
            } else {
                // a hidden activation beyond the image is the zero padding
                const NetCrop& c = ct.c[n];
                const bool inside = c.ox + x < c.img_w && c.oy + y < c.img_h;
                float r[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = acc[m][i];
                    if constexpr (MODE == kFwdRelu) {
                        v = inside ? fmaxf(v + bias[o0 + i], 0.0f) : 0.0f;
                    } else {  // through the ReLU that produced this layer's input
                        if (!(bf16_float(mask[pi * kC + o0 + i]) > 0.0f)) v = 0.0f;
                    }
                    r[i] = v;
                }
                *reinterpret_cast<uint2*>(out16 + pi * kC + o0) =
                    make_uint2(pack2(r[0], r[1]), pack2(r[2], r[3]));
            }
        }
    }
}

// ------------------------------------------------------------------ loss
// Softmax cross-entropy per pixel with a target class (pixels beyond the
// image have none); dz3 = softmax - onehot (unnormalised: every gradient is
// scaled by 1 / count at the end), stored bf16 with 32 channels (9..31
// zero).  Per workgroup: the sums of dz3 per class (b3) and per phase and
// class (P), the loss sum and the count of pixels with a target.  The sums
// of dz3 are taken in fixed point, rint(d * 2^18) in int32 (a workgroup's
// kLossPx pixels stay below 2^31), so they do not depend on the order of
// the LDS atomics and the gradient is the same on every run.
constexpr int kLossPx = 4096;
constexpr float kLossQ = 262144.0f;  // 2^18

__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ logits,
                                                   const int32_t* __restrict__ target, CropTable ct,
                                                   int S, int cw, int ch, long long total,
                                                   unsigned short* __restrict__ dz3,
                                                   float* __restrict__ partial, int region,
                                                   double* __restrict__ lossp) {
    extern __shared__ int bins[];  // 9 + 9 S^2
    __shared__ double red_l[256];
    __shared__ int red_n[256];
    for (int i = threadIdx.x; i < region; i += 256) bins[i] = 0;
    __syncthreads();
    const int per = cw * ch;
    double l = 0.0;
    int counted = 0;
    int db3[kC3];
#pragma unroll
    for (int c = 0; c < kC3; ++c) db3[c] = 0;
    for (int k = 0; k < kLossPx / 256; ++k) {
        const long long pi = static_cast<long long>(blockIdx.x) * kLossPx + k * 256 + threadIdx.x;
        if (pi >= total) break;
        const int n = static_cast<int>(pi / per), px = static_cast<int>(pi % per);
        const NetCrop& cr = ct.c[n];
        const int gx = cr.ox + px % cw, gy = cr.oy + px / cw;
        const float* lg = logits + pi * 16;
        const int t = gx < cr.img_w && gy < cr.img_h ? target[pi] : -1;
        unsigned packed[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) packed[j] = 0u;
        if (t >= 0 && t < kC3) {
            float v[kC3];
            float mx = lg[0];
#pragma unroll
            for (int c = 0; c < kC3; ++c) {
                v[c] = lg[c];
                mx = fmaxf(mx, v[c]);
            }
            float lt = 0.0f;
#pragma unroll
            for (int c = 0; c < kC3; ++c) lt = c == t ? v[c] : lt;
            float se = 0.0f;
#pragma unroll
            for (int c = 0; c < kC3; ++c) {
                v[c] = expf(v[c] - mx);
                se += v[c];
            }
            l += static_cast<double>(mx + logf(se) - lt);
            ++counted;
            const int ph = (gy % S) * S + gx % S;
            float d[kC3];
#pragma unroll
            for (int c = 0; c < kC3; ++c) {
                d[c] = v[c] / se - (c == t ? 1.0f : 0.0f);
                const int q = static_cast<int>(rintf(d[c] * kLossQ));
                db3[c] += q;
                atomicAdd(&bins[kC3 + ph * kC3 + c], q);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) packed[j] = pack2(d[2 * j], d[2 * j + 1]);
            packed[4] = pack2(d[8], 0.0f);
        }
        u32x4* o = reinterpret_cast<u32x4*>(dz3 + pi * kC);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            o[j] = u32x4{packed[4 * j], packed[4 * j + 1], packed[4 * j + 2], packed[4 * j + 3]};
    }
#pragma unroll
    for (int c = 0; c < kC3; ++c) {
        int v = db3[c];
        for (int sh = 32; sh >= 1; sh >>= 1) v += __shfl_xor(v, sh);
        if ((threadIdx.x & 63) == 0) atomicAdd(&bins[c], v);
    }
    red_l[threadIdx.x] = l;
    red_n[threadIdx.x] = counted;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red_l[threadIdx.x] += red_l[threadIdx.x + off];
            red_n[threadIdx.x] += red_n[threadIdx.x + off];
        }
        __syncthreads();
    }
    float* out = partial + static_cast<size_t>(blockIdx.x) * region;
    for (int i = threadIdx.x; i < region; i += 256) out[i] = static_cast<float>(bins[i]) / kLossQ;
    if (threadIdx.x == 0) {
        lossp[2 * blockIdx.x] = red_l[0];
        lossp[2 * blockIdx.x + 1] = static_cast<double>(red_n[0]);
    }
}

// ------------------------------------------------------- weight gradient
// dW[t][o][i] = sum over pixels p of dz[p][o] * a[p + d_t][i] (and, with a
// bias, db[o] = sum dz[p][o]) over a strip of kGW x kGStrip pixels of one
// crop, kGR rows at a time.  dz and the input (with halo) are staged in LDS
// channel-blocked: element (r, x, c) at ((r * chunks + x / 8) * 32 + c) * 8 +
// x % 8, so a lane's eight pixels of one channel are one 16-byte read; the
// one-pixel shifts of the taps are funnel shifts of neighbouring words.
// Wavefront w takes output tile m and input tile ni (two output tiles x two
// input tiles for MO = 2; for MO = 1 wavefronts 2, 3 take the odd rows and
// add into 0, 1 at the end), all nine taps.
constexpr int kGW = 64, kGR = 4, kGStrip = 32;
constexpr int kGZChunks = kGW / 8;       // dz: columns x0 .. x0 + 63
constexpr int kGAChunks = kGW / 8 + 2;   // input: columns x0 - 8 .. x0 + 71

template <int MO>
__global__ __launch_bounds__(256) void wgrad_kernel(const unsigned short* __restrict__ dz,
                                                    const unsigned short* __restrict__ a, int cw,
                                                    int ch, int cout, int cin_keep, int has_bias,
                                                    float* __restrict__ partial, int region) {
    __shared__ __align__(16) unsigned short sdz[kGR * kGZChunks * kC * 8];
    __shared__ __align__(16) unsigned short sa[(kGR + 2) * kGAChunks * kC * 8];
    const int n = blockIdx.z;
    const int x0 = blockIdx.x * kGW;
    const size_t base = static_cast<size_t>(n) * cw * ch;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int m = MO == 2 ? wave >> 1 : 0;
    const int ni = wave & 1;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;

    for (int chunk = 0; chunk < kGStrip / kGR; ++chunk) {
        const int y0 = blockIdx.y * kGStrip + chunk * kGR;
        if (y0 >= ch) break;
        for (int i = threadIdx.x; i < kGR * kGW * 4; i += 256) {
            const int q = i >> 2, part = i & 3;
            const int r = q / kGW, xx = q % kGW;
            const int x = x0 + xx, y = y0 + r;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (x < cw && y < ch)
                v = reinterpret_cast<const u32x4*>(dz + (base + static_cast<size_t>(y) * cw + x) * kC)[part];
            unsigned short* d = sdz + ((r * kGZChunks + xx / 8) * kC + part * 8) * 8 + xx % 8;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                d[(2 * j) * 8] = static_cast<unsigned short>(v[j] & 0xFFFFu);
                d[(2 * j + 1) * 8] = static_cast<unsigned short>(v[j] >> 16);
            }
        }
        for (int i = threadIdx.x; i < (kGR + 2) * kGAChunks * 8 * 4; i += 256) {
            const int q = i >> 2, part = i & 3;
            const int r = q / (kGAChunks * 8), xs = q % (kGAChunks * 8);
            const int x = x0 - 8 + xs, y = y0 - 1 + r;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (x >= 0 && y >= 0 && x < cw && y < ch)
                v = reinterpret_cast<const u32x4*>(a + (base + static_cast<size_t>(y) * cw + x) * kC)[part];
            unsigned short* d = sa + ((r * kGAChunks + xs / 8) * kC + part * 8) * 8 + xs % 8;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                d[(2 * j) * 8] = static_cast<unsigned short>(v[j] & 0xFFFFu);
                d[(2 * j + 1) * 8] = static_cast<unsigned short>(v[j] >> 16);
            }
        }
        __syncthreads();
        if (has_bias && static_cast<int>(threadIdx.x) < cout) {
            for (int r = 0; r < kGR; ++r)
                for (int c8 = 0; c8 < kGZChunks; ++c8)
                    for (int e = 0; e < 8; ++e)
                        bsum += bf16_float(sdz[((r * kGZChunks + c8) * kC + threadIdx.x) * 8 + e]);
        }
        for (int r = (MO == 2 ? 0 : wave >> 1); r < kGR; r += (MO == 2 ? 1 : 2)) {
#pragma unroll
            for (int kk = 0; kk < kGW / 32; ++kk) {
                const int c8 = kk * 4 + kq;  // chunk of this lane's 8 pixels
                const bf16x8 av = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const u32x4*>(
                                sdz + ((r * kGZChunks + c8) * kC + m * 16 + row) * 8));
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const unsigned short* srow = sa + (((r + dy) * kGAChunks) * kC + ni * 16 + row) * 8;
                    const u32x4 w1 = *reinterpret_cast<const u32x4*>(srow + (c8 + 1) * kC * 8);
                    const unsigned w0 = *reinterpret_cast<const unsigned*>(srow + c8 * kC * 8 + 6);
                    const unsigned w2 = *reinterpret_cast<const unsigned*>(srow + (c8 + 2) * kC * 8);
                    const u32x4 bl = {mid16(w1.x, w0), mid16(w1.y, w1.x), mid16(w1.z, w1.y),
                                      mid16(w1.w, w1.z)};
                    const u32x4 br = {mid16(w1.y, w1.x), mid16(w1.z, w1.y), mid16(w1.w, w1.z),
                                      mid16(w2, w1.w)};
                    acc[dy * 3 + 0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        av, __builtin_bit_cast(bf16x8, bl), acc[dy * 3 + 0], 0, 0, 0);
                    acc[dy * 3 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        av, __builtin_bit_cast(bf16x8, w1), acc[dy * 3 + 1], 0, 0, 0);
                    acc[dy * 3 + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        av, __builtin_bit_cast(bf16x8, br), acc[dy * 3 + 2], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    float* out = partial + static_cast<size_t>(blockIdx.z * gridDim.y * gridDim.x +
                                               blockIdx.y * gridDim.x + blockIdx.x) * region;
    if (MO == 1) {  // fold the odd-row wavefronts into the even-row ones
        float* red = reinterpret_cast<float*>(sa);
        if (wave >= 2)
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) red[((wave - 2) * 36 + t * 4 + i) * 64 + lane] = acc[t][i];
        __syncthreads();
        if (wave < 2)
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[t][i] += red[(wave * 36 + t * 4 + i) * 64 + lane];
    }
    if (MO == 2 || wave < 2) {
        const int in = ni * 16 + row;
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = m * 16 + kq * 4 + i;
                if (o < cout && in < cin_keep) out[(t * cout + o) * cin_keep + in] = acc[t][i];
            }
    }
    if (has_bias && static_cast<int>(threadIdx.x) < cout) out[9 * cout * cin_keep + threadIdx.x] = bsum;
}

// Sum of the partial gradients in block order, scaled by 1 / count.
struct GradRegions {
    const float* part[4];
    int start[4], size[4], nblk[4];
};

__global__ void reduce_kernel(GradRegions r, int count, const double* __restrict__ lossp,
                              int nloss, float* __restrict__ grad, double* __restrict__ loss) {
    __shared__ double s_inv;
    if (threadIdx.x == 0) {
        double tl = 0.0, tn = 0.0;
        for (int b = 0; b < nloss; ++b) {
            tl += lossp[2 * b];
            tn += lossp[2 * b + 1];
        }
        s_inv = tn > 0.0 ? 1.0 / tn : 0.0;
        if (blockIdx.x == 0 && loss) *loss = tl * s_inv;
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int j = 0;
    while (j < 3 && i >= r.start[j] + r.size[j]) ++j;
    const int li = i - r.start[j], sz = r.size[j];
    const float* p = r.part[j];
    double s = 0.0;
    for (int b = 0; b < r.nblk[j]; ++b) s += static_cast<double>(p[static_cast<size_t>(b) * sz + li]);
    grad[i] = static_cast<float>(s * s_inv);
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int count, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Training targets from converged labels: the class (dy + 1) * 3 + (dx + 1)
// of the label's cell relative to the pixel's cell; -1 if not a neighbour or
// outside the image.
__global__ void targets_kernel(CropTable ct, int S, int cw, int ch, int32_t* __restrict__ target) {
    const int px = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (px >= cw * ch) return;
    const NetCrop& c = ct.c[n];
    const int gx = c.ox + px % cw, gy = c.oy + px / cw;
    int t = -1;
    if (gx < c.img_w && gy < c.img_h) {
        const int ns_c = (c.img_w + S - 1) / S;
        const int k = c.labels[static_cast<size_t>(gy) * c.img_w + gx];
        const int dy = k / ns_c - gy / S, dx = k % ns_c - gx / S;
        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) t = (dy + 1) * 3 + (dx + 1);
    }
    target[static_cast<size_t>(n) * cw * ch + px] = t;
}

__global__ void export_logits_kernel(const float* __restrict__ lg16, long long total,
                                     float* __restrict__ out) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total * kC3) return;
    out[i] = lg16[(i / kC3) * 16 + i % kC3];
}

// ------------------------------------------ fused inference (warm start)
// The whole net plus the decoding, tile by tile (kFW x kFH output pixels),
// with every activation in LDS: the input over the tile and a 3-pixel halo,
// the first hidden layer over a 2-pixel halo, the second over a 1-pixel halo
// (regions flattened row-major and computed in N-tiles of 16 consecutive
// pixels; hidden pixels padded to 80 bytes so the 16 lanes reading one
// 16-byte chunk of 16 consecutive pixels hit distinct banks, and every tap
// is a constant offset from the lane's base address).  Activations outside
// the image are zero, which is the zero padding of every layer.  The first
// layer takes K over (tap, channel) pairs with the input stored as 4
// channels (the fourth zero): taps 0..7 in one MFMA, tap 8 in a second.
// Workgroups are persistent: each loads the weights of all three layers into
// registers once and walks tiles blockIdx.x, + gridDim.x, ...  The logits
// pass through LDS so that each lane decodes one pixel: argmax, label, and
// the pixel enters the cluster sums as in the association kernel (LDS bins,
// then one global add per non-empty bin) if it votes (its best class's
// softmax probability reaches the prepared minimum confidence); the
// workgroup holding a cell's first pixel clears that cluster's next
// accumulator.
constexpr int kFW = 32, kFH = 8;
constexpr int kXW = kFW + 6, kXH = kFH + 6;      // input region
constexpr int kA1W = kFW + 4, kA1H = kFH + 4;    // first hidden layer region
constexpr int kA2W = kFW + 2, kA2H = kFH + 2;    // second hidden layer region
constexpr int kA1N = (kA1W * kA1H + 15) / 16;    // N-tiles
constexpr int kA2N = (kA2W * kA2H + 15) / 16;
constexpr int kON = kFW * kFH / 16;
constexpr int kFusedX = kXW * kXH * 4;           // u16 elements
constexpr int kFusedA1 = kA1W * kA1H * kPS;
constexpr int kFusedA2 = kA2N * 16 * kPS;
constexpr int kFusedTab = 2 * (kFW + kFH);       // x / S, x % S, y / S, y % S
constexpr int kFusedLab = 3 * kFW * kFH;         // the tile's own CIELAB, FP32
// the decode's logits, per wavefront 64 pixels of kFusedLgStride floats (20:
// the 16-byte reads of 16 consecutive pixels hit distinct banks), in the
// first hidden layer's region after the largest bins (S = 1)
constexpr int kFusedLgStride = 20;
constexpr int kFusedMaxCells = (kFW + 2) * (kFH + 2);
constexpr int kFusedLgOff = (kFusedMaxCells * 36 + 63) / 64 * 16;  // floats
constexpr int kFT = 256;                         // threads per workgroup
constexpr int kFWaves = kFT / 64;                 // wavefronts per workgroup
constexpr int kFPerCU = 512 / kFT;                // resident workgroups per compute unit
constexpr int kXSlots = (kXW * kXH + kFT - 1) / kFT; // input pixels per thread
constexpr size_t kFusedLds = (kFusedX + kFusedA1 + kFusedA2) * sizeof(unsigned short) +
                             kFusedTab * sizeof(int) + kFusedLab * sizeof(float);
static_assert(kFPerCU * kFusedLds <= 160 * 1024, "the resident workgroups must fit one CU's LDS");
static_assert((kFusedLgOff + kFWaves * 64 * kFusedLgStride) * 4 <= kFusedA1 * 2,
              "the decode's logits fit the first hidden layer's region");

struct FusedImage {
    const float *L, *A, *B;
    int w, h, S, ns_c, ns_r;
    const float *b1, *b2, *b3, *P;
    const float* conf;  // minimum softmax probability of a voting pixel
    int32_t* labels;  // null: the decoded labels are not stored
    long long *sums_acc, *sums_next;
    int tiles_x, n_tiles;
};

// ReLU of an accumulator tile's four values packed as bf16, zero when the
// pixel lies outside the image (keep = 0; else keep = ~0).  The ReLU is
// applied to the rounded bf16 values as 16-bit integers (a negative value
// has the sign bit set, so an integer maximum with 0 clears it): the same
// result as rounding the ReLU of the FP32 value, in one packed integer
// maximum per two values, where an FP32 maximum in IEEE mode would first
// quiet each input.
// The pair is converted by one v_cvt_pk_bf16_f32 written out: through the
// vector type the compiler converts each value alone and merges the halves
// (three instructions) once the result is read as 16-bit integers.
typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned relu_bf16x2(float lo, float hi) {
    unsigned v;
    asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(v) : "v"(lo), "v"(hi));
    const i16x2 r = __builtin_elementwise_max(__builtin_bit_cast(i16x2, v), i16x2{0, 0});
    return __builtin_bit_cast(unsigned, r);
}
__device__ __forceinline__ uint2 relu_pack(const f32x4& a, unsigned keep) {
    return make_uint2(relu_bf16x2(a[0], a[1]) & keep, relu_bf16x2(a[2], a[3]) & keep);
}

__global__ __launch_bounds__(kFT, kFPerCU) void net_fused_kernel(FusedImage g, NetWeights wt) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned short* sx = reinterpret_cast<unsigned short*>(smem);
    unsigned short* sa1 = sx + kFusedX;
    unsigned short* sa2 = sa1 + kFusedA1;
    int* tab = reinterpret_cast<int*>(sa2 + kFusedA2);
    float* slab = reinterpret_cast<float*>(tab + kFusedTab);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int S = g.S;

    // ---- weights and biases, once per workgroup
    // third layer's weights in registers, one 16 x 32 fragment per tap
    bf16x8 w3r[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
        w3r[t] = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const u32x4*>(wt.W3b + (t * 16 + row) * kC + kq * 8));
    // first layer: A[o][k] with k = 4 tap + c for taps 0..7, and tap 8 alone
    bf16x8 w1[2][2], w2[9][2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kq * 8 + j, t = k >> 2, c = k & 3;
            a[j] = __builtin_bit_cast(__bf16, c < 3 ? wt.W1b[(t * kC + m * 16 + row) * kC + c]
                                                    : static_cast<unsigned short>(0));
            b[j] = __builtin_bit_cast(__bf16, (kq == 0 && j < 3) ? wt.W1b[(8 * kC + m * 16 + row) * kC + j]
                                                                  : static_cast<unsigned short>(0));
        }
        w1[m][0] = a;
        w1[m][1] = b;
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int m = 0; m < 2; ++m)
            w2[t][m] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const u32x4*>(wt.W2b + ((t * 32 + m * 16 + row) * kC + kq * 8)));
    float bias1[2][4], bias2[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bias1[m][i] = g.b1[m * 16 + kq * 4 + i];
            bias2[m][i] = g.b2[m * 16 + kq * 4 + i];
        }
    // this lane's two first-layer taps 2 kq, 2 kq + 1 as input-region offsets
    const int t0 = 2 * kq, t1 = 2 * kq + 1;
    const int xoff0 = ((t0 / 3) * kXW + t0 % 3) * 4, xoff1 = ((t1 / 3) * kXW + t1 % 3) * 4;
    const float scale = static_cast<float>(1 << kQShift);
    const float tau = *g.conf;

    // the input region of a tile, loaded one tile ahead so that its latency
    // overlaps the previous tile's work (zeros outside the image)
    float pf[kXSlots][3];
    auto prefetch = [&](int tile) {
        const int px0 = (tile % g.tiles_x) * kFW - 3, py0 = (tile / g.tiles_x) * kFH - 3;
#pragma unroll
        for (int j = 0; j < kXSlots; ++j) {
            const int q = threadIdx.x + kFT * j;
            const int gx = px0 + q % kXW, gy = py0 + q / kXW;
            pf[j][0] = pf[j][1] = pf[j][2] = 0.0f;
            if (q < kXW * kXH && gx >= 0 && gy >= 0 && gx < g.w && gy < g.h) {
                const size_t gi = static_cast<size_t>(gy) * g.w + gx;
                pf[j][0] = g.L[gi];
                pf[j][1] = g.A[gi];
                pf[j][2] = g.B[gi];
            }
        }
    };
    __builtin_amdgcn_s_waitcnt(0);  // the weights and biases are in registers
    if (static_cast<int>(blockIdx.x) < g.n_tiles) prefetch(blockIdx.x);

    for (int tile = blockIdx.x; tile < g.n_tiles; tile += gridDim.x) {
        const int x0 = (tile % g.tiles_x) * kFW, y0 = (tile / g.tiles_x) * kFH;
        // every halo pixel inside the image: no padding checks in the epilogues
        const bool interior = x0 >= 3 && y0 >= 3 && x0 + kFW + 3 <= g.w && y0 + kFH + 3 <= g.h;
        // the tile's window of grid cells and its LDS bins for the decoded
        // labels (sums of L, a, b, packed x | y | count, and the cluster of
        // each cell): in the input region when they fit (cleared during the
        // second layer, whose barrier then covers them), else in the first
        // hidden layer's region after the second layer (one more barrier)
        const int gx_lo = x0 / S - 1, gy_lo = y0 / S - 1;
        const int gx_hi = (min(x0 + kFW, g.w) - 1) / S + 1;
        const int gy_hi = (min(y0 + kFH, g.h) - 1) / S + 1;
        const int ncx = gx_hi - gx_lo + 1, ncy = gy_hi - gy_lo + 1, ncells = ncx * ncy;
        const bool early_bins = ncells * 36 <= kFusedX * static_cast<int>(sizeof(unsigned short));
        unsigned long long* const bins = reinterpret_cast<unsigned long long*>(early_bins ? sx : sa1);
        int* const kidx = reinterpret_cast<int*>(bins + 4 * ncells);
        auto init_bins = [&]() {
            for (int i = threadIdx.x; i < ncells; i += kFT) {
                const int cy = i / ncx, cx = i - cy * ncx;
                bins[i] = 0ull;
                bins[ncells + i] = 0ull;
                bins[2 * ncells + i] = 0ull;
                bins[3 * ncells + i] = 0ull;
                const int gx = gx_lo + cx, gy = gy_lo + cy;
                const bool in_grid = gx >= 0 && gy >= 0 && gx < g.ns_c && gy < g.ns_r;
                kidx[i] = in_grid ? gy * g.ns_c + gx : -1;
            }
        };
        __syncthreads();  // the previous tile's bins are flushed

        // ---- input region (bf16 L/100, a/128, b/128, 0), the tile's own
        // CIELAB in FP32, decode tables; then the next tile's loads
#pragma unroll
        for (int j = 0; j < kXSlots; ++j) {
            const int q = threadIdx.x + kFT * j;
            if (q >= kXW * kXH) continue;
            *reinterpret_cast<uint2*>(sx + q * 4) =
                make_uint2(pack2(pf[j][0] / 100.0f, pf[j][1] / 128.0f), pack2(pf[j][2] / 128.0f, 0.0f));
            const int r = q / kXW - 3, c = q % kXW - 3;
            if (r >= 0 && r < kFH && c >= 0 && c < kFW) {
                float* d = slab + (r * kFW + c) * 3;
                d[0] = pf[j][0];
                d[1] = pf[j][1];
                d[2] = pf[j][2];
            }
        }
        if (threadIdx.x < kFW) {
            const int x = x0 + threadIdx.x;
            tab[threadIdx.x] = x / S;
            tab[kFW + threadIdx.x] = x % S;
        } else if (threadIdx.x < kFW + kFH) {
            const int y = y0 + threadIdx.x - kFW;
            tab[kFW + threadIdx.x] = y / S;                 // 2 kFW + r
            tab[kFW + kFH + threadIdx.x] = y % S;           // 2 kFW + kFH + r
        }
        if (tile + static_cast<int>(gridDim.x) < g.n_tiles) prefetch(tile + gridDim.x);
        __syncthreads();

        // ---- first layer: N-tiles nt, nt + 4, ... of the wave, two at a time
        // (so that the second's loads and MFMAs overlap the first's
        // epilogue) while two remain, then a last one alone
        auto layer1 = [&](int nt, auto count) {
            constexpr int kN = decltype(count)::value;
            int pr[kN], p[kN], r[kN], c[kN];
            u32x4 bw[kN], b8[kN];
#pragma unroll
            for (int u = 0; u < kN; ++u) {
                pr[u] = (nt + u * kFWaves) * 16 + row;
                p[u] = min(pr[u], kA1W * kA1H - 1);
                r[u] = p[u] / kA1W;
                c[u] = p[u] - r[u] * kA1W;
                // input pixel (r, c) is p + 2 r: rows of the input region are
                // two pixels longer (written so, the offset is two adds; a
                // multiply-add here became a 64-bit one whose unused high
                // half waited for the next tile's pending loads)
                static_assert(kXW == kA1W + 2, "input rows are two pixels longer");
                const unsigned short* src = sx + (p[u] + 2 * r[u]) * 4;
                const uint2 v0 = *reinterpret_cast<const uint2*>(src + xoff0);
                const uint2 v1 = *reinterpret_cast<const uint2*>(src + xoff1);
                const uint2 v8 = *reinterpret_cast<const uint2*>(src + (2 * kXW + 2) * 4);
                bw[u] = u32x4{v0.x, v0.y, v1.x, v1.y};
                b8[u] = u32x4{v8.x, v8.y, 0u, 0u};
            }
            f32x4 acc[kN][2];
#pragma unroll
            for (int u = 0; u < kN; ++u)
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    acc[u][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        w1[m][0], __builtin_bit_cast(bf16x8, bw[u]),
                        f32x4{bias1[m][0], bias1[m][1], bias1[m][2], bias1[m][3]}, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < kN; ++u)
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    acc[u][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        w1[m][1], __builtin_bit_cast(bf16x8, b8[u]), acc[u][m], 0, 0, 0);
            // ReLU (the bias started the accumulator); zero outside the image
            // (tiles whose halo lies inside skip that test)
#pragma unroll
            for (int u = 0; u < kN; ++u) {
                const int gx = x0 - 2 + c[u], gy = y0 - 2 + r[u];
                const bool inside = interior || (gx >= 0 && gy >= 0 && gx < g.w && gy < g.h);
                if (pr[u] < kA1W * kA1H) {
#pragma unroll
                    for (int m = 0; m < 2; ++m)
                        *reinterpret_cast<uint2*>(sa1 + p[u] * kPS + m * 16 + kq * 4) =
                            relu_pack(acc[u][m], inside ? ~0u : 0u);
                }
            }
        };
        int nt1 = wave;
        for (; nt1 + kFWaves < kA1N; nt1 += 2 * kFWaves) layer1(nt1, std::integral_constant<int, 2>{});
        if (nt1 < kA1N) layer1(nt1, std::integral_constant<int, 1>{});
        __syncthreads();

        if (early_bins) init_bins();

        // ---- second layer over the 1-pixel halo, two N-tiles at a time
        for (int pp = wave; 2 * pp < kA2N; pp += kFWaves) {
            int pr[2], r[2], c[2];
            const unsigned short* base[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                pr[u] = (2 * pp + u) * 16 + row;
                const int p = min(pr[u], kA2W * kA2H - 1);
                r[u] = p / kA2W;
                c[u] = p - r[u] * kA2W;
                // first-layer pixel (r, c) is p + 2 r (see the first layer)
                static_assert(kA1W == kA2W + 2, "first-layer rows are two pixels longer");
                // a 24-bit multiply: a plain one became a 64-bit
                // multiply-add whose unused high half waited for pending loads
                base[u] = sa1 + __umul24(static_cast<unsigned>(p + 2 * r[u]), kPS) + kq * 8;
            }
            f32x4 acc[2][2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    acc[u][m] = f32x4{bias2[m][0], bias2[m][1], bias2[m][2], bias2[m][3]};
            // operands three taps ahead, so that each LDS read has the MFMAs
            // of two taps (eight) to arrive in
            auto operand = [&](int t, int u) {
                return __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const u32x4*>(base[u] + ((t / 3) * kA1W + t % 3) * kPS));
            };
            constexpr int kAhead = 3;
            bf16x8 bq[kAhead][2];
#pragma unroll
            for (int t = 0; t < kAhead; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) bq[t][u] = operand(t, u);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const bf16x8 b = bq[t % kAhead][u];
#pragma unroll
                    for (int m = 0; m < 2; ++m)
                        acc[u][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[t][m], b, acc[u][m], 0, 0, 0);
                    if (t + kAhead < 9) bq[t % kAhead][u] = operand(t + kAhead, u);
                }
            }
            // the schedule: six reads, then four MFMAs and two reads six
            // times, then the last twelve MFMAs (left alone, the compiler
            // keeps only two reads in flight)
            __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (2 * pp + u >= kA2N) break;
                const int gx = x0 - 1 + c[u], gy = y0 - 1 + r[u];
                const bool inside = interior || (gx >= 0 && gy >= 0 && gx < g.w && gy < g.h);
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    *reinterpret_cast<uint2*>(sa2 + pr[u] * kPS + m * 16 + kq * 4) =
                        relu_pack(acc[u][m], inside ? ~0u : 0u);
            }
        }
        __syncthreads();

        // bins of a large window: cleared now, in the first hidden layer's
        // region (the second layer has read it)
        if (!early_bins) {
            init_bins();
            __syncthreads();
        }

        // ---- third layer, then one pixel per lane: phase bias, argmax,
        // decode, accumulate.  Wave w's output N-tiles are w, w + 4, w + 8,
        // w + 12, each pixel's classes spread over four lanes (kq); a round
        // trip through LDS, written and read by the same wave (whose LDS
        // operations complete in order), gives lane (row, kq) the logits of
        // pixel (w + 4 kq) 16 + row, so that every lane decodes one pixel.
        static_assert(kON % kFWaves == 0, "output tiles split evenly over the wavefronts");
        constexpr int kPer = kON / kFWaves;
        static_assert(kPer == 4, "one decoded pixel per lane");
        const int dp = (wave + kFWaves * kq) * 16 + row;
        const int dr = dp / kFW, dc = dp % kFW;
        // the pixel's phase bias, loaded before the MFMAs
        const int ph = tab[2 * kFW + kFH + dr] * S + tab[kFW + dc];
        float pP[kC3], pB[kC3];
#pragma unroll
        for (int o = 0; o < kC3; ++o) {
            pP[o] = g.P[ph * kC3 + o];
            pB[o] = g.b3[o];
        }
        __builtin_amdgcn_sched_barrier(0);  // issued here, not next to their use
        f32x4 accs[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) accs[u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const bf16x8 w3 = w3r[t];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                // output pixel p = (wave + 4 u) * 16 + row; rows of 32 hold two N-tiles
                const int p = (wave + kFWaves * u) * 16 + row;
                static_assert(kA2W == kFW + 2, "second-layer rows are two pixels longer");
                const unsigned short* bp = sa2 + (p + 2 * (p / kFW)) * kPS + kq * 8;
                const bf16x8 b = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const u32x4*>(bp + ((t / 3) * kA2W + t % 3) * kPS));
                accs[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3, b, accs[u], 0, 0, 0);
            }
        }
        // the schedule: the operands of one tap (four reads) first, then
        // each tap's four MFMAs followed by the reads of the next tap
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
        // the phase bias has arrived: waiting here, on every path, keeps
        // the compiler from waiting for it (and for the next tile's input)
        // in the next tile's first layer
        __builtin_amdgcn_sched_barrier(0);  // the wait stays after the MFMAs
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        float* lgw = reinterpret_cast<float*>(sa1) + kFusedLgOff + wave * 64 * kFusedLgStride;
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            *reinterpret_cast<f32x4*>(lgw + (u * 16 + row) * kFusedLgStride + kq * 4) = accs[u];
        const float* mine = lgw + (kq * 16 + row) * kFusedLgStride;
        const f32x4 q0 = *reinterpret_cast<const f32x4*>(mine);
        const f32x4 q1 = *reinterpret_cast<const f32x4*>(mine + 4);
        const float q8 = mine[8];
        const float lv[kC3] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q8};
        float v[kC3];
#pragma unroll
        for (int o = 0; o < kC3; ++o) v[o] = lv[o] + (pB[o] + pP[o]);
        // best class, the lowest on ties; its softmax probability is 1 / se
        float bv = v[0];
        int bc = 0;
#pragma unroll
        for (int o = 1; o < kC3; ++o) {
            if (v[o] > bv) {
                bv = v[o];
                bc = o;
            }
        }
        float se = 0.0f;
#pragma unroll
        for (int o = 0; o < kC3; ++o) se += __expf(v[o] - bv);
        {
            const int x = x0 + dc, y = y0 + dr;
            if (x < g.w && y < g.h) {
                const int cy = min(max(tab[2 * kFW + dr] + bc / 3 - 1, 0), g.ns_r - 1);
                const int cx = min(max(tab[dc] + bc % 3 - 1, 0), g.ns_c - 1);
                if (g.labels) g.labels[static_cast<size_t>(y) * g.w + x] = cy * g.ns_c + cx;
                // the pixel votes in the first update when its best class's
                // probability reaches the prepared minimum confidence
                if (se * tau <= 1.0f) {
                    const int cell = (cy - gy_lo) * ncx + (cx - gx_lo);
                    const float* lab = slab + dp * 3;
                    // |v| 2^18 < 2^31 for every CIELAB value
                    const int ql = static_cast<int>(rintf(lab[0] * scale));
                    const int qa = static_cast<int>(rintf(lab[1] * scale));
                    const int qb = static_cast<int>(rintf(lab[2] * scale));
                    atomicAdd(bins + cell, static_cast<unsigned long long>(static_cast<long long>(ql)));
                    atomicAdd(bins + ncells + cell,
                              static_cast<unsigned long long>(static_cast<long long>(qa)));
                    atomicAdd(bins + 2 * ncells + cell,
                              static_cast<unsigned long long>(static_cast<long long>(qb)));
                    atomicAdd(bins + 3 * ncells + cell,
                              static_cast<unsigned long long>(dc) |
                                  (static_cast<unsigned long long>(dr) << 20) | (1ull << 40));
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < ncells; i += kFT) {
            // the tile holding a cell's first pixel clears that cluster's
            // next accumulator
            const int k = kidx[i];
            if (k >= 0) {
                const int cx = k % g.ns_c, cy = k / g.ns_c;
                if ((cx * S) / kFW == x0 / kFW && (cy * S) / kFH == y0 / kFH) {
                    long long* z = g.sums_next + static_cast<size_t>(k) * kSumStride;
                    for (int j = 0; j < kSumStride; ++j) z[j] = 0;
                }
            }
            const unsigned long long pk = bins[3 * ncells + i];
            const long long cnt = static_cast<long long>(pk >> 40);
            if (cnt == 0) continue;
            unsigned long long* sm = reinterpret_cast<unsigned long long*>(
                g.sums_acc + static_cast<size_t>(kidx[i]) * kSumStride);
            atomicAdd(sm + 0, bins[i]);
            atomicAdd(sm + 1, bins[ncells + i]);
            atomicAdd(sm + 2, bins[2 * ncells + i]);
            atomicAdd(sm + 3, static_cast<unsigned long long>(static_cast<long long>(pk & 0xFFFFFull) + cnt * x0));
            atomicAdd(sm + 4, static_cast<unsigned long long>(
                                  static_cast<long long>((pk >> 20) & 0xFFFFFull) + cnt * y0));
            atomicAdd(sm + 5, static_cast<unsigned long long>(cnt));
        }
    }
}

// ------------------------------------------------------------ host side

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct NetWs {
    unsigned short *x, *a1, *a2, *dz3, *dz2;  // dz1 reuses dz3, dz2 the logits
    float* logits;
    NetWeights wt;
    float *part_w1, *part_w2, *part_w3, *part_loss;
    double* lossp;
    int nb_grad, nb_loss, loss_region;
};

int grad_blocks(int n, int cw, int ch) {
    return ((cw + kGW - 1) / kGW) * ((ch + kGStrip - 1) / kGStrip) * n;
}
int loss_blocks(long long total) { return static_cast<int>((total + kLossPx - 1) / kLossPx); }

// Workspace parts by mode: kWeights (the bf16 weight copies), kForward
// (+ activations and logits), kTraining (+ gradients and partial sums).
enum NetMode { kWeights = 0, kForward = 1, kTraining = 2 };

size_t net_layout(int n, int cw, int ch, int S, int mode, NetWs* nw, char* base) {
    const size_t P = static_cast<size_t>(n) * cw * ch;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    NetWs w{};
    w.wt.W1b = reinterpret_cast<unsigned short*>(take(9 * kC * kC * 2));
    w.wt.W2b = reinterpret_cast<unsigned short*>(take(9 * kC * kC * 2));
    w.wt.W3b = reinterpret_cast<unsigned short*>(take(9 * 16 * kC * 2));
    w.wt.W2t = reinterpret_cast<unsigned short*>(take(9 * kC * kC * 2));
    w.wt.W3t = reinterpret_cast<unsigned short*>(take(9 * kC * kC * 2));
    if (mode >= kForward) {
        w.x = reinterpret_cast<unsigned short*>(take(P * kC * 2));
        w.a1 = reinterpret_cast<unsigned short*>(take(P * kC * 2));
        w.a2 = reinterpret_cast<unsigned short*>(take(P * kC * 2));
        w.logits = reinterpret_cast<float*>(take(P * 16 * sizeof(float)));
        w.dz2 = reinterpret_cast<unsigned short*>(w.logits);
    }
    if (mode >= kTraining) {
        w.dz3 = reinterpret_cast<unsigned short*>(take(P * kC * 2));
        w.nb_grad = grad_blocks(n, cw, ch);
        w.nb_loss = loss_blocks(static_cast<long long>(P));
        w.loss_region = kC3 + kC3 * S * S;
        w.part_w1 = reinterpret_cast<float*>(take(static_cast<size_t>(w.nb_grad) * (kOffW2 - kOffW1) * 4));
        w.part_w2 = reinterpret_cast<float*>(take(static_cast<size_t>(w.nb_grad) * (kOffW3 - kOffW2) * 4));
        w.part_w3 = reinterpret_cast<float*>(take(static_cast<size_t>(w.nb_grad) * (kOffB3 - kOffW3) * 4));
        w.part_loss = reinterpret_cast<float*>(take(static_cast<size_t>(w.nb_loss) * w.loss_region * 4));
        w.lossp = reinterpret_cast<double*>(take(static_cast<size_t>(w.nb_loss) * 2 * sizeof(double)));
    }
    if (nw) *nw = w;
    return off;
}

bool shape_ok(int n, int cw, int ch, int S) {
    return n >= 1 && n <= kMaxCrops && cw >= 1 && ch >= 1 && cw <= (1 << 16) && ch <= (1 << 16) &&
           static_cast<long long>(n) * cw * ch < (1ll << 31) / kC && S >= 1 && S <= kMaxS;
}

bool device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

bool crops_ok(const slic_net_crop* crops, int n, bool need_lab, bool need_labels) {
    if (!crops) return false;
    for (int i = 0; i < n; ++i) {
        const slic_net_crop& c = crops[i];
        if (c.img_w < 1 || c.img_h < 1 || c.ox < 0 || c.oy < 0 || c.ox >= c.img_w || c.oy >= c.img_h)
            return false;
        if (static_cast<long long>(c.img_w) * c.img_h >= (1ll << 31)) return false;
        if (need_lab && (!device_ptr(c.d_L) || !device_ptr(c.d_a) || !device_ptr(c.d_b))) return false;
        if (need_labels && !device_ptr(c.d_labels)) return false;
    }
    return true;
}

CropTable crop_table(const slic_net_crop* crops, int n) {
    CropTable t;
    std::memset(&t, 0, sizeof(t));
    for (int i = 0; i < n; ++i) {
        t.c[i] = NetCrop{crops[i].d_L, crops[i].d_a, crops[i].d_b, crops[i].d_labels,
                         crops[i].img_w, crops[i].img_h, crops[i].ox, crops[i].oy};
    }
    return t;
}

hipError_t enqueue_forward(const NetWs& nw, const CropTable& ct, int n, int cw, int ch, int S,
                           const float* params, hipStream_t s) {
    {
        KernelTimer t("net_prepare", s);
        prepare_kernel<<<(9 * kC * kC + 255) / 256, 256, 0, s>>>(params, nw.wt, 0, nullptr,
                                                                  nullptr, 0.0f);
    }
    const int per = cw * ch;
    {
        KernelTimer t("net_input", s);
        input_kernel<<<dim3((per + 255) / 256, n), 256, 0, s>>>(ct, cw, ch, nw.x);
    }
    const dim3 grid((cw + kTW - 1) / kTW, (ch + kTRows - 1) / kTRows, n);
    {
        KernelTimer t("net_conv1", s);
        conv_kernel<2, kFwdRelu><<<grid, 256, 0, s>>>(nw.x, nw.wt.W1b, params + kOffB1, nullptr, ct,
                                                      S, cw, ch, nullptr, nw.a1, nullptr);
    }
    {
        KernelTimer t("net_conv2", s);
        conv_kernel<2, kFwdRelu><<<grid, 256, 0, s>>>(nw.a1, nw.wt.W2b, params + kOffB2, nullptr, ct,
                                                      S, cw, ch, nullptr, nw.a2, nullptr);
    }
    {
        KernelTimer t("net_conv3", s);
        conv_kernel<1, kFwdLogits><<<grid, 256, 0, s>>>(nw.a2, nw.wt.W3b, params + kOffB3,
                                                        params + kOffP, ct, S, cw, ch, nullptr,
                                                        nullptr, nw.logits);
    }
    return hipGetLastError();
}

hipError_t enqueue_backward(const NetWs& nw, const CropTable& ct, int n, int cw, int ch, int S,
                            const int32_t* target, float* grad, double* loss, hipStream_t s) {
    const long long total = static_cast<long long>(n) * cw * ch;
    {
        KernelTimer t("net_loss", s);
        loss_kernel<<<nw.nb_loss, 256, nw.loss_region * sizeof(int), s>>>(
            nw.logits, target, ct, S, cw, ch, total, nw.dz3, nw.part_loss, nw.loss_region, nw.lossp);
    }
    const dim3 ggrid((cw + kGW - 1) / kGW, (ch + kGStrip - 1) / kGStrip, n);
    const dim3 cgrid((cw + kTW - 1) / kTW, (ch + kTRows - 1) / kTRows, n);
    {
        KernelTimer t("net_wgrad3", s);
        wgrad_kernel<1><<<ggrid, 256, 0, s>>>(nw.dz3, nw.a2, cw, ch, kC3, kC, 0, nw.part_w3,
                                              kOffB3 - kOffW3);
    }
    {
        KernelTimer t("net_dgrad3", s);
        conv_kernel<2, kBwdMasked><<<cgrid, 256, 0, s>>>(nw.dz3, nw.wt.W3t, nullptr, nullptr, ct, S,
                                                         cw, ch, nw.a2, nw.dz2, nullptr);
    }
    {
        KernelTimer t("net_wgrad2", s);
        wgrad_kernel<2><<<ggrid, 256, 0, s>>>(nw.dz2, nw.a1, cw, ch, kC, kC, 1, nw.part_w2,
                                              kOffW3 - kOffW2);
    }
    unsigned short* dz1 = nw.dz3;
    {
        KernelTimer t("net_dgrad2", s);
        conv_kernel<2, kBwdMasked><<<cgrid, 256, 0, s>>>(nw.dz2, nw.wt.W2t, nullptr, nullptr, ct, S,
                                                         cw, ch, nw.a1, dz1, nullptr);
    }
    {
        KernelTimer t("net_wgrad1", s);
        wgrad_kernel<2><<<ggrid, 256, 0, s>>>(dz1, nw.x, cw, ch, kC, 3, 1, nw.part_w1,
                                              kOffW2 - kOffW1);
    }
    GradRegions r;
    r.part[0] = nw.part_w1;
    r.start[0] = kOffW1;
    r.size[0] = kOffW2 - kOffW1;
    r.nblk[0] = nw.nb_grad;
    r.part[1] = nw.part_w2;
    r.start[1] = kOffW2;
    r.size[1] = kOffW3 - kOffW2;
    r.nblk[1] = nw.nb_grad;
    r.part[2] = nw.part_w3;
    r.start[2] = kOffW3;
    r.size[2] = kOffB3 - kOffW3;
    r.nblk[2] = nw.nb_grad;
    r.part[3] = nw.part_loss;
    r.start[3] = kOffB3;
    r.size[3] = nw.loss_region;
    r.nblk[3] = nw.nb_loss;
    const int count = kOffP + kC3 * S * S;
    {
        KernelTimer t("net_reduce", s);
        reduce_kernel<<<(count + 255) / 256, 256, 0, s>>>(r, count, nw.lossp, nw.nb_loss, grad, loss);
    }
    return hipGetLastError();
}

}  // namespace

// A prepared net: the bf16 weight copies followed by the FP32 parameter
// vector, sized for the largest S so that a phase index never leaves it,
// and then the decode's minimum confidence (one float).
constexpr int kMaxParams = kOffP + kC3 * kMaxS * kMaxS;

size_t prepared_layout(NetWeights* wt, float** params, char* base) {
    NetWs nw;
    const size_t off = net_layout(1, 1, 1, 1, kWeights, &nw, base);
    if (wt) *wt = nw.wt;
    if (params) *params = base ? reinterpret_cast<float*>(base + off) : nullptr;
    return off + align_up(static_cast<size_t>(kMaxParams + 1) * sizeof(float));
}

hipError_t launch_warm_start(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                             const void* d_net, hipStream_t s, bool store_labels) {
    NetWeights wt;
    float* params;
    prepared_layout(&wt, &params, static_cast<char*>(const_cast<void*>(d_net)));
    const size_t ring = static_cast<size_t>(g.K) * kSumStride;
    const int tiles_x = (w + kFW - 1) / kFW;
    const int n_tiles = tiles_x * ((h + kFH - 1) / kFH);
    FusedImage f{ws.L, ws.A, ws.B, w, h, g.S, g.ns_c, g.ns_r,
                 params + kOffB1, params + kOffB2, params + kOffB3, params + kOffP,
                 params + kMaxParams, store_labels ? ws.labels : nullptr, ws.sums,
                 ws.sums + ring, tiles_x, n_tiles};
    // persistent workgroups, kFPerCU per compute unit (their LDS fits that often)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    const int grid = n_tiles < kFPerCU * cus ? n_tiles : kFPerCU * cus;
    // above 64 KiB of dynamic LDS needs the opt-in, once per device (setting
    // it twice from racing threads is harmless)
    static std::atomic<unsigned long long> lds_set{0ull};
    const unsigned long long bit = dev < 64 ? 1ull << dev : 0ull;
    if (!bit || !(lds_set.load(std::memory_order_acquire) & bit)) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(net_fused_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(kFusedLds));
        if (e != hipSuccess) return e;
        lds_set.fetch_or(bit, std::memory_order_acq_rel);
    }
    KernelTimer t("net_fused", s);
    net_fused_kernel<<<grid, kFT, kFusedLds, s>>>(f, wt);
    return hipGetLastError();
}

bool warm_supported(int32_t S) { return S >= 1 && S <= kMaxS; }

// The step S each prepared buffer was filled for, per (device, address).
namespace {
std::mutex g_prepared_mu;
std::map<std::pair<int, uintptr_t>, int32_t> g_prepared;
}  // namespace

void record_prepared(const void* d_net, int32_t S) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(g_prepared_mu);
    g_prepared[std::make_pair(dev, reinterpret_cast<uintptr_t>(d_net))] = S;
}

int32_t prepared_step(const void* d_net) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(g_prepared_mu);
    auto it = g_prepared.find(std::make_pair(dev, reinterpret_cast<uintptr_t>(d_net)));
    return it == g_prepared.end() ? 0 : it->second;
}

}  // namespace slic

using namespace slic;

extern "C" {

size_t slic_net_prepared_bytes(void) { return prepared_layout(nullptr, nullptr, nullptr); }

int slic_net_prepare(int32_t S, const float* d_params, float min_confidence, void* d_net,
                     void* hip_stream) {
    if (S < 1 || S > kMaxS || !(min_confidence >= 0.0f) || !std::isfinite(min_confidence) ||
        !device_ptr(d_params) || !device_ptr(d_net) ||
        reinterpret_cast<uintptr_t>(d_net) % kAlign != 0)
        return SLIC_EINVAL;
    NetWeights wt;
    float* params;
    prepared_layout(&wt, &params, static_cast<char*>(d_net));
    const int count = kOffP + kC3 * S * S;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int n = count > 9 * kC * kC ? count : 9 * kC * kC;
    prepare_kernel<<<(n + 255) / 256, 256, 0, s>>>(d_params, wt, count, params,
                                                   params + kMaxParams, min_confidence);
    if (hipGetLastError() != hipSuccess) return SLIC_EHIP;
    record_prepared(d_net, S);
    return SLIC_OK;
}

int32_t slic_net_param_count(int32_t S) {
    if (S < 1 || S > kMaxS) return 0;
    return kOffP + kC3 * S * S;
}

size_t slic_net_workspace_bytes(int32_t n_crops, int32_t crop_w, int32_t crop_h, int32_t S) {
    if (!shape_ok(n_crops, crop_w, crop_h, S)) return 0;
    return net_layout(n_crops, crop_w, crop_h, S, kTraining, nullptr, nullptr);
}

int slic_net_forward(const slic_net_crop* crops, int32_t n_crops, int32_t crop_w, int32_t crop_h,
                     int32_t S, const float* d_params, float* d_logits, void* hip_stream,
                     void* d_ws, size_t ws_bytes) {
    if (!shape_ok(n_crops, crop_w, crop_h, S) || !crops_ok(crops, n_crops, true, false))
        return SLIC_EINVAL;
    if (!device_ptr(d_params) || !device_ptr(d_logits) || !device_ptr(d_ws) ||
        reinterpret_cast<uintptr_t>(d_ws) % kAlign != 0 ||
        ws_bytes < net_layout(n_crops, crop_w, crop_h, S, kForward, nullptr, nullptr))
        return SLIC_EINVAL;
    NetWs nw;
    net_layout(n_crops, crop_w, crop_h, S, kForward, &nw, static_cast<char*>(d_ws));
    const CropTable ct = crop_table(crops, n_crops);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (enqueue_forward(nw, ct, n_crops, crop_w, crop_h, S, d_params, s) != hipSuccess) return SLIC_EHIP;
    const long long total = static_cast<long long>(n_crops) * crop_w * crop_h;
    {
        KernelTimer t("net_export", s);
        export_logits_kernel<<<static_cast<unsigned>((total * kC3 + 255) / 256), 256, 0, s>>>(
            nw.logits, total, d_logits);
    }
    return hipGetLastError() == hipSuccess ? SLIC_OK : SLIC_EHIP;
}

int slic_net_loss_grad(const slic_net_crop* crops, int32_t n_crops, int32_t crop_w, int32_t crop_h,
                       int32_t S, const float* d_params, const int32_t* d_target, float* d_grad,
                       double* d_loss, void* hip_stream, void* d_ws, size_t ws_bytes) {
    if (!shape_ok(n_crops, crop_w, crop_h, S) || !crops_ok(crops, n_crops, true, false))
        return SLIC_EINVAL;
    if (!device_ptr(d_params) || !device_ptr(d_target) || !device_ptr(d_grad) || !device_ptr(d_ws) ||
        (d_loss && !device_ptr(d_loss)) || reinterpret_cast<uintptr_t>(d_ws) % kAlign != 0 ||
        ws_bytes < net_layout(n_crops, crop_w, crop_h, S, kTraining, nullptr, nullptr))
        return SLIC_EINVAL;
    NetWs nw;
    net_layout(n_crops, crop_w, crop_h, S, kTraining, &nw, static_cast<char*>(d_ws));
    const CropTable ct = crop_table(crops, n_crops);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (enqueue_forward(nw, ct, n_crops, crop_w, crop_h, S, d_params, s) != hipSuccess) return SLIC_EHIP;
    if (enqueue_backward(nw, ct, n_crops, crop_w, crop_h, S, d_target, d_grad, d_loss, s) != hipSuccess)
        return SLIC_EHIP;
    return SLIC_OK;
}

int slic_net_targets(const slic_net_crop* crops, int32_t n_crops, int32_t crop_w, int32_t crop_h,
                     int32_t S, int32_t* d_target, void* hip_stream) {
    if (!shape_ok(n_crops, crop_w, crop_h, S) || !crops_ok(crops, n_crops, false, true) ||
        !device_ptr(d_target))
        return SLIC_EINVAL;
    const CropTable ct = crop_table(crops, n_crops);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int per = crop_w * crop_h;
    targets_kernel<<<dim3((per + 255) / 256, n_crops), 256, 0, s>>>(ct, S, crop_w, crop_h, d_target);
    return hipGetLastError() == hipSuccess ? SLIC_OK : SLIC_EHIP;
}

int slic_net_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, int32_t count,
                  int32_t step, float lr, float beta1, float beta2, float eps, void* hip_stream) {
    if (count < 1 || step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) || !device_ptr(d_params) ||
        !device_ptr(d_grad) || !device_ptr(d_m) || !device_ptr(d_v))
        return SLIC_EINVAL;
    const float c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), step));
    const float c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), step));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    adam_kernel<<<(count + 255) / 256, 256, 0, s>>>(d_params, d_grad, d_m, d_v, count, lr, beta1,
                                                    beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? SLIC_OK : SLIC_EHIP;
}

}  // extern "C"
