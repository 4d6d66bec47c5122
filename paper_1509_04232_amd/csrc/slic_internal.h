// Internal declarations of libslic (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "slic.h"

namespace slic {

// Colour values enter the centre sums as exact integers rint(v * 2^18).
// |v| < 108 for every sRGB colour, so |q| < 2^25 and a 64-lane sum of q
// fits in int32.
constexpr int kQShift = 18;

// Centres are stored padded to 8 floats (L, a, b, x, y, -, -, -) so a
// centre is two aligned 16-byte loads.
constexpr int kCenStride = 8;

// Per-cluster accumulators: sum qL, qa, qb, x, y and the pixel count.
constexpr int kSumStride = 6;

struct Grid {
    int32_t S, ns_c, ns_r, K;
    float w;      // m / S in FP32, the factor of d_xy in Eq. 1
    int32_t space;  // colour planes: 0 CIELAB, 1 XYZ x 100, 2 the RGB bytes
    int32_t dist;   // 0 Eq. 1, 1 the squared-sum form d_lab^2 + w^2 d_xy^2
};

struct Workspace {
    float *L, *A, *B;    // planar CIELAB, N each
    int32_t* labels;     // N, cluster index per pixel
    float* cen;          // K x kCenStride
    int32_t* counts;     // K, pixels per centre at the last update
    long long* sums;     // 3 x K x kSumStride, a ring of accumulators
    int32_t *ccl0, *ccl1, *ccl2, *ccl3;  // N each, connectivity scratch
    int32_t* scan;       // block totals of the connectivity prefix sum
    double* partial;     // per-block energy partial sums
    long long* ctl;      // convergence control: residual ring [3], stop flag, iterations
    int32_t n_scan_blocks, n_energy_blocks;
};

// Byte offsets of the workspace parts; returns the total size.
size_t workspace_layout(int32_t width, int32_t height, const Grid& g, Workspace* ws, char* base);

// Number of prefix-sum tiles the connectivity pass uses for n pixels.
int scan_tiles_for(int n);

// Launch wrappers (each returns the hipError_t of its launches).
// CIELAB conversion of the image into ws.L/A/B fused with the seeding of
// every centre (and the clearing of its count and first accumulators).
struct LabSeedImage {
    const uint8_t* rgb;
    int w, h, pitch, channels;
    float *L, *A, *B;
    int S, ns_c, ns_r, perturb, space;
    float* cen;
    int32_t* counts;
    long long* sums;  // first accumulator buffer
    int tiles_x;      // conversion tiles per row
};
struct LabSeedTileMap {
    const LabSeedImage* images;
    const int* tile_image;
    const int* tile_first;
};
hipError_t launch_lab_seed(const uint8_t* rgb, int32_t w, int32_t h, int32_t pitch,
                           int32_t channels, const Workspace& ws, const Grid& grid, int perturb,
                           hipStream_t s);
hipError_t launch_lab_seed_batch(const LabSeedTileMap& map, int total_tiles, hipStream_t s);
LabSeedImage lab_seed_image(const uint8_t* rgb, int32_t w, int32_t h, int32_t pitch,
                            int32_t channels, const Workspace& ws, const Grid& grid, int perturb);
int lab_seed_tile_w();
int lab_seed_tile_h();
// Per-image description of an association launch (constant across
// launches; the launch number t selects the accumulator buffers).
struct AssignImage {
    const float* L;
    const float* A;
    const float* B;
    int w, h, S, ns_c, ns_r, K;
    float wgt;
    float* cen;        // K x kCenStride: centres used by the last launch
    int32_t* counts;   // K
    int32_t* labels;   // N
    long long* sums;   // ring of 3 x K x kSumStride accumulators
    int tiles_x;       // workgroup tiles per row (for the launch's variant)
};

// Batch launches: workgroup b works on tile b - tile_first[i] of image
// i = tile_image[b], described by images[i] (all in device memory).
struct AssignTileMap {
    const AssignImage* images;
    const int* tile_image;
    const int* tile_first;
};

// Convergence stop (Section 2): with ctl set, association launch t also sums
// the quantised L1 shift of the centres it updates into ctl[t % 3]; launch t
// of a run that began at t_first exits at once if a previous launch stopped
// the run (ctl[3] != 0) or if t > t_first and the shift of launch t - 1 is
// below limit, in which case it sets ctl[3] = 1 and ctl[4] = t - t_first.
struct Converge {
    long long* ctl;
    long long limit;
    long long t_first;
};
hipError_t launch_converge_reset(long long* ctl, hipStream_t s);
hipError_t launch_converge_result(const long long* ctl, int32_t max_iters, int32_t* out,
                                  hipStream_t s);

// Association launch number t (0: the first, with the seeds as centres;
// t >= 1 also completes the centre update of the previous launch).
// variant: launch shape 1..assign_variant_count(); an unsupported value
// falls back to assign_default_variant.  store_labels false: the labels are
// not written (a launch that another association launch follows before
// anything reads them).
hipError_t launch_assign(const Workspace& ws, int32_t w, int32_t h, const Grid& g, int64_t t,
                         int variant, hipStream_t s, const Converge* cv = nullptr,
                         bool store_labels = true);
// Association launch t as the last one before the connectivity clean-up:
// it also writes the clean-up's tile-local components (ws.ccl0, ws.ccl3,
// ws.ccl1, the connectivity pass's first step), so launch_connectivity then
// runs with local_done.  Only where assign_final_ccl_supported (the launch
// has the 1 x 4 shape, whose tiles are the clean-up's 32 x 32 tiles).
bool assign_final_ccl_supported(int32_t w, int32_t h, int32_t S);
hipError_t launch_assign_final_ccl(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                                  int64_t t, hipStream_t s);
hipError_t launch_assign_batch(const AssignTileMap& map, int total_tiles, int min_S, int64_t t,
                               int variant, int dist, hipStream_t s, bool store_labels = true);
AssignImage assign_image(const Workspace& ws, int32_t w, int32_t h, const Grid& g, int variant);
bool assign_tiles(int variant, int32_t w, int32_t h, int* tiles_x, int* tiles_y);
int assign_variant_count();
bool assign_variant_shape(int variant, int* vec, int* rows, int* tile_w, int* tile_h);
bool assign_variant_supported(int variant, int32_t w, int32_t h, int32_t S);
int assign_default_variant(int32_t w, int32_t h, int32_t S);
hipError_t launch_energy(const Workspace& ws, int32_t w, int32_t h, const Grid& g, double* out,
                         hipStream_t s);
// local_done: the final association launch already wrote the tile-local
// components (launch_assign_final_ccl), so the first pass is skipped.
hipError_t launch_connectivity(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                               int32_t min_segment, int32_t* labels_out, int32_t* n_segments,
                               hipStream_t s, bool local_done = false);

// Connectivity of one image: device pointers into its workspace and sizes.
struct CclImage {
    const int32_t* labels;  // association labels (input)
    int32_t* out;           // final labels (may be `labels`)
    int32_t* comp;          // local roots, then component roots
    int32_t* size;          // component sizes
    int32_t* rank;          // survivor ranks and join links
    int32_t* lroot;         // local roots (index inside the 32 x 32 tile)
    int32_t* block_count;   // survivors per run of 1024 pixels
    int32_t* n_segments;    // the segment count (may be null)
    int w, h;
    long long S2;           // S * S
    int min_segment;
    int tiles_x;            // 32 x 32 tiles per row
    int nmerge;             // runs of 1024 pixels
};

// Batch connectivity: workgroup b of a tile pass works on tile
// b - tile_first[i] of image i = tile_image[b]; of a pixel-run pass on run
// b - blk_first[i] of image i = blk_image[b] (all in device memory).
struct CclMap {
    const CclImage* images;
    const int* tile_image;
    const int* tile_first;
    const int* blk_image;
    const int* blk_first;
};

CclImage ccl_image(const Workspace& ws, int32_t w, int32_t h, const Grid& g, int32_t min_segment,
                   int32_t* labels_out, int32_t* n_segments);
int ccl_tiles_for(int32_t w, int32_t h);
// Whether an image can take part in a batched connectivity launch (its
// segment numbering fits the relabel pass's own scan).
bool ccl_batch_supported(int32_t w, int32_t h);
hipError_t launch_connectivity_batch(const CclMap& map, int total_tiles, int total_blocks,
                                     int max_nmerge, hipStream_t s);
// Section 3's stray-pixel filter on `labels` in place (ws.ccl0 as the second
// buffer), `passes` passes.
hipError_t launch_stray_filter(const Workspace& ws, int32_t w, int32_t h, int32_t* labels,
                               int32_t passes, hipStream_t s);
// A given first association (after launch_lab_seed): ws.labels from
// `given` (entries outside [0, K) become the pixel's own grid cell), the
// valid entries accumulated into the first accumulators, the second
// cleared, so that association launch 1 starts from them.
hipError_t launch_import_labels(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                                const int32_t* given, hipStream_t s);
// Centres float[K][5] from the caller into the workspace (stride kCenStride).
hipError_t launch_import_centres(const Workspace& ws, const Grid& g, const float* in,
                                 hipStream_t s);
hipError_t launch_export_centres(const Workspace& ws, const Grid& g, float* out, int32_t* counts,
                                 hipStream_t s);

// Learned warm start (net.hip).  warm_supported: the net handles step S.
// launch_warm_start: after launch_lab_seed, runs the prepared net d_net on
// ws.L/A/B, writes the decoded labels to ws.labels (unless store_labels is
// false: association rounds follow before anything reads them), accumulates
// them into the first accumulator buffer (as association launch 0 would)
// and clears the second, so that association launch 1 starts from the
// net's labels.
bool warm_supported(int32_t S);
// slic_net_prepare records the step S each prepared buffer holds (per
// device and address); prepared_step returns it, 0 for a buffer it never
// prepared on the current device.
void record_prepared(const void* d_net, int32_t S);
int32_t prepared_step(const void* d_net);
hipError_t launch_warm_start(const Workspace& ws, int32_t w, int32_t h, const Grid& g,
                             const void* d_net, hipStream_t s, bool store_labels = true);

// Kernel timing: while enabled, a KernelTimer brackets a launch with HIP
// events on the launch stream.
bool timing_enabled();
class KernelTimer {
  public:
    KernelTimer(const char* name, hipStream_t s);
    ~KernelTimer();

  private:
    const char* name_;
    hipStream_t s_;
    void* start_;
};

}  // namespace slic

struct slic_ctx {
    slic_params p;
    slic::Grid g;
    slic::Workspace ws;
    hipStream_t stream;
    int device;
    int variant;    // association launch variant
    int64_t t;      // association launches so far
    int state;      // 0: k-means state valid, 1: connectivity done, 2: poisoned,
                    // 3: stopped by the convergence rule (final)
};
