// A given first association (slic_init_from_labels): the labels go to the
// workspace and their pixels into the first centre accumulators, in the
// fixed-point form the association kernel uses (Section 3, updating the
// cluster centre).
#include "slic_internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace slic {
namespace {

// Each thread takes kImportRun pixels of one row: it stores their labels (an entry outside [0, K) stands for the
// pixel's own grid cell) and adds every run of equal valid labels to the
// first accumulators in one go (fixed-point colour sums, as the
// association does; integer adds, so the order does not matter).  The
// threads of the first K * kSumStride also clear the second accumulators.
constexpr int kImportRun = 8;

__global__ __launch_bounds__(256) void import_labels_kernel(
    const int32_t* __restrict__ given, int w, int h, int S, int ns_c, int K,
    const float* __restrict__ L, const float* __restrict__ A, const float* __restrict__ B,
    int32_t* __restrict__ labels, long long* __restrict__ sums0, long long* __restrict__ sums1) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < static_cast<long long>(K) * kSumStride) sums1[t] = 0;
    const int per_row = (w + kImportRun - 1) / kImportRun;
    if (t >= static_cast<long long>(per_row) * h) return;
    const int y = static_cast<int>(t / per_row);
    const int xb = static_cast<int>(t % per_row) * kImportRun;
    const int xe = min(xb + kImportRun, w);
    const float scale = static_cast<float>(1 << kQShift);
    int run_k = -1, run_x0 = 0, run_n = 0;
    long long ql = 0, qa = 0, qb = 0;
    auto flush = [&]() {
        if (run_n == 0) return;
        unsigned long long* sm =
            reinterpret_cast<unsigned long long*>(sums0 + static_cast<size_t>(run_k) * kSumStride);
        const long long n = run_n;
        atomicAdd(sm + 0, static_cast<unsigned long long>(ql));
        atomicAdd(sm + 1, static_cast<unsigned long long>(qa));
        atomicAdd(sm + 2, static_cast<unsigned long long>(qb));
        atomicAdd(sm + 3, static_cast<unsigned long long>(n * run_x0 + n * (n - 1) / 2));
        atomicAdd(sm + 4, static_cast<unsigned long long>(n * y));
        atomicAdd(sm + 5, static_cast<unsigned long long>(n));
    };
    for (int x = xb; x < xe; ++x) {
        const size_t i = static_cast<size_t>(y) * w + x;
        const int k = given[i];
        const bool valid = k >= 0 && k < K;
        labels[i] = valid ? k : (y / S) * ns_c + x / S;
        if (!valid || k != run_k || x != run_x0 + run_n) {
            flush();
            run_n = 0;
            ql = qa = qb = 0;
            run_k = valid ? k : -1;
            run_x0 = x;
        }
        if (!valid) continue;
        ql += static_cast<long long>(rintf(L[i] * scale));
        qa += static_cast<long long>(rintf(A[i] * scale));
        qb += static_cast<long long>(rintf(B[i] * scale));
        ++run_n;
    }
    flush();
}

}  // namespace

hipError_t launch_import_labels(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                                const int32_t* given, hipStream_t s) {
    const long long threads = std::max(static_cast<long long>((w + kImportRun - 1) / kImportRun) * h,
                                       static_cast<long long>(g.K) * kSumStride);
    const size_t ring = static_cast<size_t>(g.K) * kSumStride;
    KernelTimer t("import_labels", s);
    import_labels_kernel<<<static_cast<unsigned>((threads + 255) / 256), 256, 0, s>>>(
        given, w, h, g.S, g.ns_c, g.K, ws.L, ws.A, ws.B, ws.labels, ws.sums, ws.sums + ring);
    return hipGetLastError();
}

}  // namespace slic
