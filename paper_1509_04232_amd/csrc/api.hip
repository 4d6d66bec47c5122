// The C ABI of libslic: validation, workspace layout, contexts and the
// control flow of Section 4's listing (convert, initialise the centres,
// associate, then n x (update, associate), then optionally enforce
// connectivity), all enqueued on the caller's stream.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "slic_internal.h"

namespace slic {

// ---------------------------------------------------------------- timing

namespace {
struct TimedLaunch {
    const char* name;
    hipEvent_t start, stop;
};
bool g_timing = false;
std::vector<TimedLaunch> g_launches;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool timing_enabled() { return g_timing; }

KernelTimer::KernelTimer(const char* name, hipStream_t s) : name_(name), s_(s), start_(nullptr) {
    if (!g_timing) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) == hipSuccess) start_ = e;
}

KernelTimer::~KernelTimer() {
    if (!start_) return;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s_) == hipSuccess)
        g_launches.push_back({name_, static_cast<hipEvent_t>(start_), e});
}

// ------------------------------------------------------------- workspace

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int energy_blocks_for(int n) { return (n + 255) / 256; }
}  // namespace

size_t workspace_layout(int32_t width, int32_t height, const Grid& g, Workspace* ws, char* base) {
    const size_t n = static_cast<size_t>(width) * height;
    const size_t K = static_cast<size_t>(g.K);
    const int nscan = scan_tiles_for(static_cast<int>(n));
    const int nenergy = energy_blocks_for(static_cast<int>(n));
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    Workspace w{};
    w.L = reinterpret_cast<float*>(take(n * sizeof(float)));
    w.A = reinterpret_cast<float*>(take(n * sizeof(float)));
    w.B = reinterpret_cast<float*>(take(n * sizeof(float)));
    w.labels = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
    w.cen = reinterpret_cast<float*>(take(K * kCenStride * sizeof(float)));
    w.counts = reinterpret_cast<int32_t*>(take(K * sizeof(int32_t)));
    w.sums = reinterpret_cast<long long*>(take(3 * K * kSumStride * sizeof(long long)));
    w.ccl0 = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
    w.ccl1 = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
    w.ccl2 = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
    w.ccl3 = reinterpret_cast<int32_t*>(take(n * sizeof(int32_t)));
    w.scan = reinterpret_cast<int32_t*>(take(static_cast<size_t>(nscan) * sizeof(int32_t)));
    w.partial = reinterpret_cast<double*>(take(static_cast<size_t>(nenergy) * sizeof(double)));
    w.ctl = reinterpret_cast<long long*>(take(8 * sizeof(long long)));
    w.n_scan_blocks = nscan;
    w.n_energy_blocks = nenergy;
    if (ws) *ws = w;
    return off;
}

// ------------------------------------------------------------ validation

namespace {

constexpr int32_t kMaxSide = 1 << 24;  // pixel coordinates exact in FP32

// Integer grid step (Section 2: S = sqrt(N/K)), rounded to nearest.
bool compute_grid(const slic_params* p, Grid* g) {
    int32_t S = p->S;
    if (S <= 0) {
        const double n = static_cast<double>(p->width) * static_cast<double>(p->height);
        const double s = std::floor(std::sqrt(n / static_cast<double>(p->K)) + 0.5);
        S = s < 1.0 ? 1 : (s > 2147483647.0 ? 2147483647 : static_cast<int32_t>(s));
    }
    g->S = S;
    g->ns_c = static_cast<int32_t>((static_cast<int64_t>(p->width) + S - 1) / S);
    g->ns_r = static_cast<int32_t>((static_cast<int64_t>(p->height) + S - 1) / S);
    g->K = g->ns_c * g->ns_r;
    g->w = p->m / static_cast<float>(S);
    g->space = (p->flags & SLIC_COLOR_XYZ) ? 1 : (p->flags & SLIC_COLOR_RGB) ? 2 : 0;
    g->dist = (p->flags & SLIC_DISTANCE_SQUARED) ? 1 : 0;
    return true;
}

bool params_ok(const slic_params* p) {
    if (!p) return false;
    if (p->width < 1 || p->height < 1 || p->width > kMaxSide || p->height > kMaxSide) return false;
    if (static_cast<int64_t>(p->width) * p->height >= (static_cast<int64_t>(1) << 31) / 2)
        return false;
    if (p->channels != 3 && p->channels != 4) return false;
    if (static_cast<int64_t>(p->pitch) < static_cast<int64_t>(p->width) * p->channels) return false;
    if (p->S < 0 || (p->S == 0 && p->K < 1)) return false;
    if (!std::isfinite(p->m) || p->m < 0.0f) return false;
    // (m / S) d_xy, and its square, stay finite for every pixel and centre
    // of the image (d_xy below the diagonal plus one cell)
    {
        Grid g;
        compute_grid(p, &g);
        const double diag = std::sqrt(static_cast<double>(p->width) * p->width +
                                      static_cast<double>(p->height) * p->height) + 2.0 * g.S;
        if (static_cast<double>(p->m) / g.S * diag > 1e15) return false;
    }
    if (p->flags & ~(SLIC_PERTURB_SEEDS | SLIC_COLOR_XYZ | SLIC_COLOR_RGB | SLIC_DISTANCE_SQUARED))
        return false;
    if ((p->flags & SLIC_COLOR_XYZ) && (p->flags & SLIC_COLOR_RGB)) return false;
    if (p->min_segment < 0) return false;
    return true;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

// 0: device memory, SLIC_EINVAL: not device memory, SLIC_EHIP: runtime error
int check_device_ptr(const void* p) {
    if (!p) return SLIC_EINVAL;
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e == hipErrorNoDevice || e == hipErrorInsufficientDriver || e == hipErrorNotInitialized) {
        (void)hipGetLastError();
        return SLIC_EHIP;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return SLIC_EINVAL;
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) return SLIC_EINVAL;
    return SLIC_OK;
}

int check_buffers(const void* rgb, const void* ws) {
    int rc = check_device_ptr(rgb);
    if (rc) return rc;
    return check_device_ptr(ws);
}

// Association launch c->t.  With ccl set and *ccl true (the last launch
// before the connectivity clean-up), the launch that also finds the
// tile-local components where the image allows its shape; *ccl then says
// whether it did.  store: whether the labels are written (a launch that
// another association follows before anything reads them skips them).
hipError_t associate(slic_ctx* c, bool* ccl, bool store) {
    const slic_params& p = c->p;
    if (ccl && *ccl && !assign_final_ccl_supported(p.width, p.height, c->g.S)) *ccl = false;
    if (ccl && *ccl) return launch_assign_final_ccl(c->ws, p.width, p.height, c->g, c->t, c->stream);
    return launch_assign(c->ws, p.width, p.height, c->g, c->t, c->variant, c->stream, nullptr,
                         store);
}

// Section 4's listing up to the first association (ccl, store: as in
// associate, for a first association that is also the last, or that rounds
// follow at once).
hipError_t enqueue_init(slic_ctx* c, const uint8_t* rgb, bool* ccl = nullptr, bool store = true) {
    const slic_params& p = c->p;
    hipError_t e = launch_lab_seed(rgb, p.width, p.height, p.pitch, p.channels, c->ws, c->g,
                                   (p.flags & SLIC_PERTURB_SEEDS) ? 1 : 0, c->stream);
    if (e != hipSuccess) return e;
    c->t = 0;
    e = associate(c, ccl, store);
    if (e == hipSuccess) c->t = 1;
    return e;
}

// n rounds of (update, associate): each association launch also completes
// the previous launch's centre update (ccl: as in associate, for the last
// of them; untouched when n is 0).  Only the last launch writes the labels.
hipError_t enqueue_iterations(slic_ctx* c, int32_t n, bool* ccl = nullptr) {
    for (int32_t i = 0; i < n; ++i) {
        hipError_t e = associate(c, i == n - 1 ? ccl : nullptr, i == n - 1);
        if (e != hipSuccess) return e;
        ++c->t;
    }
    return hipSuccess;
}

int fail(slic_ctx* c) {
    if (c) c->state = 2;
    return SLIC_EHIP;
}

// Process-wide choice of association variant per (width, height, S),
// filled by slic_set_assign_variant or slic_autotune.
std::mutex g_variant_mu;
std::map<std::tuple<int32_t, int32_t, int32_t>, int> g_variant;

int resolve_variant(int32_t w, int32_t h, int32_t S) {
    {
        std::lock_guard<std::mutex> lock(g_variant_mu);
        auto it = g_variant.find(std::make_tuple(w, h, S));
        if (it != g_variant.end() && assign_variant_supported(it->second, w, h, S)) return it->second;
    }
    return assign_default_variant(w, h, S);
}

void bind(slic_ctx* c, const slic_params* p, void* d_ws, void* stream) {
    c->p = *p;
    compute_grid(p, &c->g);
    workspace_layout(p->width, p->height, c->g, &c->ws, static_cast<char*>(d_ws));
    c->stream = static_cast<hipStream_t>(stream);
    c->state = 0;
    c->variant = resolve_variant(p->width, p->height, c->g.S);
    c->t = 0;
    c->device = 0;
}

}  // namespace
}  // namespace slic

// ------------------------------------------------------------------ batch

struct slic_batch {
    int n = 0;
    std::vector<slic_params> params;
    std::vector<slic::Grid> grids;
    std::vector<slic::Workspace> ws;
    std::vector<const uint8_t*> rgb;
    std::vector<int32_t*> labels;
    int32_t* n_segments = nullptr;
    int n_iters = 0, enforce = 0, variant = 0, use_graph = 0;
    int min_S = 0;
    // device tables inside the caller's workspace
    slic::LabSeedImage* lab_images = nullptr;
    int* lab_tile_image = nullptr;
    int* lab_tile_first = nullptr;
    int lab_tiles = 0;
    slic::AssignImage* asg_images = nullptr;
    int* asg_tile_image = nullptr;
    int* asg_tile_first = nullptr;
    int asg_tiles = 0, asg_tiles_cap = 0;
    slic::CclImage* ccl_images = nullptr;
    int* ccl_tile_image = nullptr;
    int* ccl_tile_first = nullptr;
    int* ccl_blk_image = nullptr;
    int* ccl_blk_first = nullptr;
    int ccl_tiles = 0, ccl_blocks = 0, ccl_max_nmerge = 0;
    int ccl_batched = 0;  // every image fits the batched connectivity launches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int state = 0;  // 0 ok, 2 poisoned
};

namespace slic {
namespace {

int batch_variant_ok(const slic_batch* b, int v) {
    for (int i = 0; i < b->n; ++i)
        if (!assign_variant_supported(v, b->params[i].width, b->params[i].height, b->grids[i].S))
            return 0;
    return 1;
}

// Bytes of the batch workspace: every image's own workspace, then the tables.
size_t batch_layout(const slic_params* p, int32_t n, slic_batch* b, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* q = base ? base + off : nullptr;
        off += align_up(bytes);
        return q;
    };
    int lab_tiles = 0, asg_cap = 0, ccl_tiles = 0, ccl_blocks = 0;
    for (int i = 0; i < n; ++i) {
        ccl_tiles += ccl_tiles_for(p[i].width, p[i].height);
        ccl_blocks += scan_tiles_for(p[i].width * p[i].height);
        Grid g;
        compute_grid(p + i, &g);
        Workspace w{};
        const size_t bytes = workspace_layout(p[i].width, p[i].height, g, &w, nullptr);
        char* region = take(bytes);
        if (b) {
            workspace_layout(p[i].width, p[i].height, g, &w, region);
            b->grids.push_back(g);
            b->ws.push_back(w);
        }
        lab_tiles += ((p[i].width + lab_seed_tile_w() - 1) / lab_seed_tile_w()) *
                     ((p[i].height + lab_seed_tile_h() - 1) / lab_seed_tile_h());
        int most = 0;  // the variant with the smallest tiles has the most
        for (int v = 1; v <= assign_variant_count(); ++v) {
            int tx = 0, ty = 0;
            assign_tiles(v, p[i].width, p[i].height, &tx, &ty);
            most = std::max(most, tx * ty);
        }
        asg_cap += most;
    }
    char* li = take(sizeof(LabSeedImage) * n);
    char* lt = take(sizeof(int) * lab_tiles);
    char* lf = take(sizeof(int) * n);
    char* ai = take(sizeof(AssignImage) * n);
    char* at = take(sizeof(int) * asg_cap);
    char* af = take(sizeof(int) * n);
    char* ci = take(sizeof(CclImage) * n);
    char* ct = take(sizeof(int) * ccl_tiles);
    char* cf = take(sizeof(int) * n);
    char* cb = take(sizeof(int) * ccl_blocks);
    char* cbf = take(sizeof(int) * n);
    if (b) {
        b->ccl_images = reinterpret_cast<CclImage*>(ci);
        b->ccl_tile_image = reinterpret_cast<int*>(ct);
        b->ccl_tile_first = reinterpret_cast<int*>(cf);
        b->ccl_blk_image = reinterpret_cast<int*>(cb);
        b->ccl_blk_first = reinterpret_cast<int*>(cbf);
        b->lab_images = reinterpret_cast<LabSeedImage*>(li);
        b->lab_tile_image = reinterpret_cast<int*>(lt);
        b->lab_tile_first = reinterpret_cast<int*>(lf);
        b->lab_tiles = lab_tiles;
        b->asg_images = reinterpret_cast<AssignImage*>(ai);
        b->asg_tile_image = reinterpret_cast<int*>(at);
        b->asg_tile_first = reinterpret_cast<int*>(af);
        b->asg_tiles_cap = asg_cap;
    }
    return off;
}

// Upload the association tables for variant v (synchronous copies).
hipError_t batch_upload_assign(slic_batch* b, int v) {
    std::vector<AssignImage> imgs(b->n);
    std::vector<int> first(b->n), tile_image;
    for (int i = 0; i < b->n; ++i) {
        imgs[i] = assign_image(b->ws[i], b->params[i].width, b->params[i].height, b->grids[i], v);
        int tx = 0, ty = 0;
        assign_tiles(v, b->params[i].width, b->params[i].height, &tx, &ty);
        first[i] = static_cast<int>(tile_image.size());
        tile_image.insert(tile_image.end(), static_cast<size_t>(tx) * ty, i);
    }
    b->asg_tiles = static_cast<int>(tile_image.size());
    b->variant = v;
    hipError_t e = hipMemcpy(b->asg_images, imgs.data(), sizeof(AssignImage) * b->n,
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->asg_tile_image, tile_image.data(), sizeof(int) * tile_image.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->asg_tile_first, first.data(), sizeof(int) * b->n, hipMemcpyHostToDevice);
    return e;
}

hipError_t batch_upload_lab(slic_batch* b) {
    std::vector<LabSeedImage> imgs(b->n);
    std::vector<int> first(b->n), tile_image;
    for (int i = 0; i < b->n; ++i) {
        const slic_params& p = b->params[i];
        imgs[i] = lab_seed_image(b->rgb[i], p.width, p.height, p.pitch, p.channels, b->ws[i],
                                 b->grids[i], (p.flags & SLIC_PERTURB_SEEDS) ? 1 : 0);
        const int tiles = imgs[i].tiles_x * ((p.height + lab_seed_tile_h() - 1) / lab_seed_tile_h());
        first[i] = static_cast<int>(tile_image.size());
        tile_image.insert(tile_image.end(), static_cast<size_t>(tiles), i);
    }
    hipError_t e = hipMemcpy(b->lab_images, imgs.data(), sizeof(LabSeedImage) * b->n,
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->lab_tile_image, tile_image.data(), sizeof(int) * tile_image.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->lab_tile_first, first.data(), sizeof(int) * b->n, hipMemcpyHostToDevice);
    return e;
}

// Connectivity tables: every image's descriptor and the maps from
// workgroups to (image, tile) and (image, run of 1024 pixels).
hipError_t batch_upload_ccl(slic_batch* b) {
    std::vector<CclImage> imgs(b->n);
    std::vector<int> tfirst(b->n), bfirst(b->n), tile_image, blk_image;
    b->ccl_batched = 1;
    b->ccl_max_nmerge = 0;
    for (int i = 0; i < b->n; ++i) {
        const slic_params& p = b->params[i];
        imgs[i] = ccl_image(b->ws[i], p.width, p.height, b->grids[i], p.min_segment, b->labels[i],
                            b->n_segments ? b->n_segments + i : nullptr);
        if (!ccl_batch_supported(p.width, p.height)) b->ccl_batched = 0;
        b->ccl_max_nmerge = std::max(b->ccl_max_nmerge, imgs[i].nmerge);
        tfirst[i] = static_cast<int>(tile_image.size());
        tile_image.insert(tile_image.end(), static_cast<size_t>(ccl_tiles_for(p.width, p.height)), i);
        bfirst[i] = static_cast<int>(blk_image.size());
        blk_image.insert(blk_image.end(), static_cast<size_t>(imgs[i].nmerge), i);
    }
    b->ccl_tiles = static_cast<int>(tile_image.size());
    b->ccl_blocks = static_cast<int>(blk_image.size());
    hipError_t e = hipMemcpy(b->ccl_images, imgs.data(), sizeof(CclImage) * b->n,
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->ccl_tile_image, tile_image.data(), sizeof(int) * tile_image.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->ccl_tile_first, tfirst.data(), sizeof(int) * b->n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->ccl_blk_image, blk_image.data(), sizeof(int) * blk_image.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->ccl_blk_first, bfirst.data(), sizeof(int) * b->n, hipMemcpyHostToDevice);
    return e;
}

// The whole pipeline for every image: one conversion+seeding launch,
// 1 + n_iters association launches, then the connectivity passes (each one
// launch over every image when all of them fit the batched passes).
hipError_t batch_enqueue(const slic_batch* b, hipStream_t s) {
    const LabSeedTileMap lmap{b->lab_images, b->lab_tile_image, b->lab_tile_first};
    hipError_t e = launch_lab_seed_batch(lmap, b->lab_tiles, s);
    const AssignTileMap amap{b->asg_images, b->asg_tile_image, b->asg_tile_first};
    for (int t = 0; e == hipSuccess && t <= b->n_iters; ++t)  // only the last writes labels
        e = launch_assign_batch(amap, b->asg_tiles, b->min_S, t, b->variant, b->grids[0].dist, s,
                                t == b->n_iters);
    if (e == hipSuccess && b->enforce && b->ccl_batched) {
        const CclMap cmap{b->ccl_images, b->ccl_tile_image, b->ccl_tile_first, b->ccl_blk_image,
                          b->ccl_blk_first};
        return launch_connectivity_batch(cmap, b->ccl_tiles, b->ccl_blocks, b->ccl_max_nmerge, s);
    }
    for (int i = 0; e == hipSuccess && b->enforce && i < b->n; ++i) {
        Workspace w = b->ws[i];
        w.labels = b->labels[i];
        e = launch_connectivity(w, b->params[i].width, b->params[i].height, b->grids[i],
                                b->params[i].min_segment, b->labels[i],
                                b->n_segments ? b->n_segments + i : nullptr, s);
    }
    return e;
}

void batch_drop_graph(slic_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Capture the pipeline into a graph on a private default-priority stream.
hipError_t batch_capture(slic_batch* b) {
    batch_drop_graph(b);
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t ee = batch_enqueue(b, cs);
        e = hipStreamEndCapture(cs, &b->graph);
        if (ee != hipSuccess) e = ee;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) batch_drop_graph(b);
    return e;
}

// The whole listing into a workspace that holds at least
// slic_workspace_bytes(p) bytes (arguments already validated).
int enqueue_segment(const slic_params* p, const uint8_t* d_rgb, int32_t n_iters, int32_t enforce,
                    int32_t* d_labels, float* d_centres, double* d_energy, int32_t* d_n_segments,
                    void* hip_stream, void* d_ws) {
    slic_ctx c;
    bind(&c, p, d_ws, hip_stream);
    c.ws.labels = d_labels;  // associate straight into the caller's buffer
    // the last association also finds the tile-local components, if it can
    bool local_done = enforce != 0;
    if (enqueue_init(&c, d_rgb, n_iters == 0 ? &local_done : nullptr, n_iters == 0) != hipSuccess)
        return SLIC_EHIP;
    if (enqueue_iterations(&c, n_iters, &local_done) != hipSuccess) return SLIC_EHIP;
    if (d_energy &&
        launch_energy(c.ws, p->width, p->height, c.g, d_energy, c.stream) != hipSuccess)
        return SLIC_EHIP;
    if (d_centres && launch_export_centres(c.ws, c.g, d_centres, nullptr, c.stream) != hipSuccess)
        return SLIC_EHIP;
    if (enforce && launch_connectivity(c.ws, p->width, p->height, c.g, p->min_segment, d_labels,
                                       d_n_segments, c.stream, local_done) != hipSuccess)
        return SLIC_EHIP;
    return SLIC_OK;
}

}  // namespace
}  // namespace slic

// --------------------------------------------- allocation-free workspace

// The workspace of slic_segment_noalloc: one array per device, loaded with
// the library's code object and held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in); it uses the device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[SLIC_NOALLOC_MAX_WORKSPACE];

namespace slic {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The address of `scratch` on the current device, looked up once per device
// with that device current.
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace slic

using namespace slic;

extern "C" {

size_t slic_workspace_bytes(const slic_params* p) {
    if (!params_ok(p)) return 0;
    Grid g;
    compute_grid(p, &g);
    return workspace_layout(p->width, p->height, g, nullptr, nullptr);
}

int slic_grid(const slic_params* p, int32_t* S, int32_t* ns_c, int32_t* ns_r) {
    if (!params_ok(p)) return SLIC_EINVAL;
    Grid g;
    compute_grid(p, &g);
    if (S) *S = g.S;
    if (ns_c) *ns_c = g.ns_c;
    if (ns_r) *ns_r = g.ns_r;
    return SLIC_OK;
}

int slic_init(slic_ctx** out, const slic_params* p, const uint8_t* d_rgb, void* hip_stream,
              void* d_ws, size_t ws_bytes) {
    if (!out || !params_ok(p) || !d_rgb || !d_ws || !aligned(d_ws)) return SLIC_EINVAL;
    *out = nullptr;
    if (ws_bytes < slic_workspace_bytes(p)) return SLIC_EINVAL;
    int rc = check_buffers(d_rgb, d_ws);
    if (rc) return rc;
    slic_ctx* c = new (std::nothrow) slic_ctx;
    if (!c) return SLIC_ENOMEM;
    bind(c, p, d_ws, hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess || enqueue_init(c, d_rgb) != hipSuccess) {
        delete c;
        return SLIC_EHIP;
    }
    *out = c;
    return SLIC_OK;
}

int slic_init_from_centres(slic_ctx** out, const slic_params* p, const uint8_t* d_rgb,
                           const float* d_centres, void* hip_stream, void* d_ws, size_t ws_bytes) {
    if (!out || !params_ok(p) || !d_rgb || !d_centres || !d_ws || !aligned(d_ws))
        return SLIC_EINVAL;
    *out = nullptr;
    if (ws_bytes < slic_workspace_bytes(p)) return SLIC_EINVAL;
    int rc = check_buffers(d_rgb, d_ws);
    if (rc == SLIC_OK) rc = check_device_ptr(d_centres);
    if (rc) return rc;
    slic_ctx* c = new (std::nothrow) slic_ctx;
    if (!c) return SLIC_ENOMEM;
    bind(c, p, d_ws, hip_stream);
    const slic_params& q = c->p;
    // the conversion kernel also seeds (and clears the counts and first
    // accumulators); the given centres then replace the seeds
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess)
        e = launch_lab_seed(d_rgb, q.width, q.height, q.pitch, q.channels, c->ws, c->g, 0, c->stream);
    if (e == hipSuccess) e = launch_import_centres(c->ws, c->g, d_centres, c->stream);
    if (e == hipSuccess) {
        c->t = 0;
        e = launch_assign(c->ws, q.width, q.height, c->g, c->t, c->variant, c->stream);
    }
    if (e != hipSuccess) {
        delete c;
        return SLIC_EHIP;
    }
    c->t = 1;
    *out = c;
    return SLIC_OK;
}

int slic_init_from_labels(slic_ctx** out, const slic_params* p, const uint8_t* d_rgb,
                          const int32_t* d_labels0, void* hip_stream, void* d_ws, size_t ws_bytes) {
    if (!out || !params_ok(p) || !d_rgb || !d_labels0 || !d_ws || !aligned(d_ws))
        return SLIC_EINVAL;
    *out = nullptr;
    if (ws_bytes < slic_workspace_bytes(p)) return SLIC_EINVAL;
    int rc = check_buffers(d_rgb, d_ws);
    if (rc == SLIC_OK) rc = check_device_ptr(d_labels0);
    if (rc) return rc;
    slic_ctx* c = new (std::nothrow) slic_ctx;
    if (!c) return SLIC_ENOMEM;
    bind(c, p, d_ws, hip_stream);
    const slic_params& q = c->p;
    // conversion and seeding (which clears the first accumulators), then the
    // given labels as association launch 0
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess)
        e = launch_lab_seed(d_rgb, q.width, q.height, q.pitch, q.channels, c->ws, c->g,
                            (q.flags & SLIC_PERTURB_SEEDS) ? 1 : 0, c->stream);
    if (e == hipSuccess) e = launch_import_labels(c->ws, q.width, q.height, c->g, d_labels0, c->stream);
    if (e != hipSuccess) {
        delete c;
        return SLIC_EHIP;
    }
    c->t = 1;
    *out = c;
    return SLIC_OK;
}

int slic_iterate(slic_ctx* c, int32_t n_iters) {
    if (!c || n_iters < 0) return SLIC_EINVAL;
    if (c->state != 0) return SLIC_ESTATE;
    return enqueue_iterations(c, n_iters) == hipSuccess ? SLIC_OK : fail(c);
}

int slic_iterate_converge(slic_ctx* c, int32_t max_iters, float threshold,
                          int32_t* d_iters_done) {
    if (!c || max_iters < 0 || !(threshold >= 0.0f) || !std::isfinite(threshold))
        return SLIC_EINVAL;
    if (d_iters_done && check_device_ptr(d_iters_done) != SLIC_OK) return SLIC_EINVAL;
    if (c->state != 0) return SLIC_ESTATE;
    const double q = std::ldexp(static_cast<double>(threshold), kQShift);
    if (q * static_cast<double>(c->g.K) > 4.0e18) return SLIC_EINVAL;
    const Converge cv{c->ws.ctl, std::llrint(q) * static_cast<long long>(c->g.K), c->t};
    if (launch_converge_reset(c->ws.ctl, c->stream) != hipSuccess) return fail(c);
    for (int32_t i = 0; i < max_iters; ++i) {
        if (launch_assign(c->ws, c->p.width, c->p.height, c->g, c->t, c->variant, c->stream, &cv) !=
            hipSuccess)
            return fail(c);
        ++c->t;
    }
    if (d_iters_done && launch_converge_result(c->ws.ctl, max_iters, d_iters_done, c->stream) !=
                            hipSuccess)
        return fail(c);
    c->state = 3;
    return SLIC_OK;
}

int slic_enforce_connectivity(slic_ctx* c, int32_t* d_n_segments) {
    if (!c) return SLIC_EINVAL;
    if (c->state != 0 && c->state != 3) return SLIC_ESTATE;
    if (launch_connectivity(c->ws, c->p.width, c->p.height, c->g, c->p.min_segment, c->ws.labels,
                            d_n_segments, c->stream) != hipSuccess)
        return fail(c);
    c->state = 1;
    return SLIC_OK;
}

int slic_filter_stray(slic_ctx* c, int32_t passes) {
    if (!c || passes < 0) return SLIC_EINVAL;
    if (c->state != 0 && c->state != 3) return SLIC_ESTATE;
    if (launch_stray_filter(c->ws, c->p.width, c->p.height, c->ws.labels, passes, c->stream) !=
        hipSuccess)
        return fail(c);
    c->state = 1;
    return SLIC_OK;
}

int slic_get_labels(const slic_ctx* c, int32_t* d_labels) {
    if (!c || !d_labels) return SLIC_EINVAL;
    if (c->state == 2) return SLIC_ESTATE;
    const size_t bytes = static_cast<size_t>(c->p.width) * c->p.height * sizeof(int32_t);
    if (hipMemcpyAsync(d_labels, c->ws.labels, bytes, hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
        return fail(const_cast<slic_ctx*>(c));
    return SLIC_OK;
}

int slic_get_centres(const slic_ctx* c, float* d_centres, int32_t* d_counts) {
    if (!c || !d_centres) return SLIC_EINVAL;
    if (c->state == 2) return SLIC_ESTATE;
    if (launch_export_centres(c->ws, c->g, d_centres, d_counts, c->stream) != hipSuccess)
        return fail(const_cast<slic_ctx*>(c));
    return SLIC_OK;
}

int slic_get_lab(const slic_ctx* c, float* d_L, float* d_a, float* d_b) {
    if (!c || !d_L || !d_a || !d_b) return SLIC_EINVAL;
    if (c->state == 2) return SLIC_ESTATE;
    const size_t bytes = static_cast<size_t>(c->p.width) * c->p.height * sizeof(float);
    const float* src[3] = {c->ws.L, c->ws.A, c->ws.B};
    float* dst[3] = {d_L, d_a, d_b};
    for (int j = 0; j < 3; ++j)
        if (hipMemcpyAsync(dst[j], src[j], bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return fail(const_cast<slic_ctx*>(c));
    return SLIC_OK;
}

int slic_energy(const slic_ctx* c, double* d_out) {
    if (!c || !d_out) return SLIC_EINVAL;
    if (c->state != 0 && c->state != 3) return SLIC_ESTATE;
    if (launch_energy(c->ws, c->p.width, c->p.height, c->g, d_out, c->stream) != hipSuccess)
        return fail(const_cast<slic_ctx*>(c));
    return SLIC_OK;
}

int slic_segment(const slic_params* p, const uint8_t* d_rgb, int32_t n_iters, int32_t enforce,
                 int32_t* d_labels, float* d_centres, double* d_energy, int32_t* d_n_segments,
                 void* hip_stream, void* d_ws, size_t ws_bytes) {
    if (!params_ok(p) || !d_rgb || !d_labels || !d_ws || !aligned(d_ws) || n_iters < 0)
        return SLIC_EINVAL;
    if (ws_bytes < slic_workspace_bytes(p)) return SLIC_EINVAL;
    int rc = check_buffers(d_rgb, d_ws);
    if (rc) return rc;
    if ((rc = check_device_ptr(d_labels)) != 0) return rc;
    return enqueue_segment(p, d_rgb, n_iters, enforce, d_labels, d_centres, d_energy,
                           d_n_segments, hip_stream, d_ws);
}

int slic_segment_noalloc(const slic_params* p, const uint8_t* d_rgb, int32_t n_iters,
                         int32_t enforce, int32_t* d_labels, float* d_centres, double* d_energy,
                         int32_t* d_n_segments, void* hip_stream) {
    if (!params_ok(p) || !d_rgb || !d_labels || n_iters < 0) return SLIC_EINVAL;
    if (slic_workspace_bytes(p) > static_cast<size_t>(SLIC_NOALLOC_MAX_WORKSPACE))
        return SLIC_EINVAL;
    int rc = check_device_ptr(d_rgb);
    if (rc == SLIC_OK) rc = check_device_ptr(d_labels);
    if (rc) return rc;
    void* ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return SLIC_EHIP;
    return enqueue_segment(p, d_rgb, n_iters, enforce, d_labels, d_centres, d_energy,
                           d_n_segments, hip_stream, ws);
}

namespace {

// slic_init with the net's decoded labels as the first association (store:
// whether the decoded labels are written; rounds that follow at once make
// them dead).
hipError_t enqueue_warm_init(slic_ctx* c, const uint8_t* rgb, const void* d_net,
                             bool store = true) {
    const slic_params& p = c->p;
    hipError_t e = launch_lab_seed(rgb, p.width, p.height, p.pitch, p.channels, c->ws, c->g,
                                   (p.flags & SLIC_PERTURB_SEEDS) ? 1 : 0, c->stream);
    if (e != hipSuccess) return e;
    c->t = 0;
    e = launch_warm_start(c->ws, p.width, p.height, c->g, d_net, c->stream, store);
    if (e == hipSuccess) c->t = 1;
    return e;
}

int check_warm_args(const slic_params* p, const uint8_t* d_rgb, const void* d_net, void* d_ws,
                    size_t ws_bytes) {
    if (!params_ok(p) || !d_rgb || !d_net || !d_ws || !aligned(d_ws) || !aligned(d_net))
        return SLIC_EINVAL;
    Grid g;
    compute_grid(p, &g);
    if (!warm_supported(g.S) || g.space != 0 || g.dist != 0 || ws_bytes < slic_workspace_bytes(p))
        return SLIC_EINVAL;
    int rc = check_buffers(d_rgb, d_ws);
    if (rc == SLIC_OK) rc = check_device_ptr(d_net);
    if (rc) return rc;
    // the phase bias is indexed with the image's S: the net must have been
    // prepared for that S
    return prepared_step(d_net) == g.S ? SLIC_OK : SLIC_EINVAL;
}

}  // namespace

size_t slic_warm_workspace_bytes(const slic_params* p) {
    if (!params_ok(p)) return 0;
    Grid g;
    compute_grid(p, &g);
    return warm_supported(g.S) && g.space == 0 && g.dist == 0 ? slic_workspace_bytes(p) : 0;
}

int slic_warm_init(slic_ctx** out, const slic_params* p, const uint8_t* d_rgb, const void* d_net,
                   void* hip_stream, void* d_ws, size_t ws_bytes) {
    if (!out) return SLIC_EINVAL;
    *out = nullptr;
    int rc = check_warm_args(p, d_rgb, d_net, d_ws, ws_bytes);
    if (rc) return rc;
    slic_ctx* c = new (std::nothrow) slic_ctx;
    if (!c) return SLIC_ENOMEM;
    bind(c, p, d_ws, hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess || enqueue_warm_init(c, d_rgb, d_net) != hipSuccess) {
        delete c;
        return SLIC_EHIP;
    }
    *out = c;
    return SLIC_OK;
}

int slic_warm_segment(const slic_params* p, const uint8_t* d_rgb, const void* d_net,
                      int32_t n_iters, int32_t enforce, int32_t* d_labels, float* d_centres,
                      double* d_energy, int32_t* d_n_segments, void* hip_stream, void* d_ws,
                      size_t ws_bytes) {
    if (n_iters < 0 || !d_labels) return SLIC_EINVAL;
    int rc = check_warm_args(p, d_rgb, d_net, d_ws, ws_bytes);
    if (rc) return rc;
    if ((rc = check_device_ptr(d_labels)) != 0) return rc;
    slic_ctx c;
    bind(&c, p, d_ws, hip_stream);
    c.ws.labels = d_labels;
    if (enqueue_warm_init(&c, d_rgb, d_net, n_iters == 0) != hipSuccess) return SLIC_EHIP;
    // with rounds, the last association also finds the tile-local components
    bool local_done = enforce != 0 && n_iters > 0;
    if (enqueue_iterations(&c, n_iters, &local_done) != hipSuccess) return SLIC_EHIP;
    if (d_energy &&
        launch_energy(c.ws, p->width, p->height, c.g, d_energy, c.stream) != hipSuccess)
        return SLIC_EHIP;
    if (d_centres && launch_export_centres(c.ws, c.g, d_centres, nullptr, c.stream) != hipSuccess)
        return SLIC_EHIP;
    if (enforce && launch_connectivity(c.ws, p->width, p->height, c.g, p->min_segment, d_labels,
                                       d_n_segments, c.stream, local_done) != hipSuccess)
        return SLIC_EHIP;
    return SLIC_OK;
}

void slic_destroy(slic_ctx* c) { delete c; }

int32_t slic_assign_variants(void) { return assign_variant_count(); }

int slic_assign_variant_info(int32_t variant, int32_t* vec, int32_t* rows, int32_t* tile_w,
                             int32_t* tile_h) {
    int v = 0, r = 0, tw = 0, th = 0;
    if (!assign_variant_shape(variant, &v, &r, &tw, &th)) return SLIC_EINVAL;
    if (vec) *vec = v;
    if (rows) *rows = r;
    if (tile_w) *tile_w = tw;
    if (tile_h) *tile_h = th;
    return SLIC_OK;
}

int slic_set_assign_variant(int32_t width, int32_t height, int32_t S, int32_t variant) {
    if (width < 1 || height < 1 || S < 1) return SLIC_EINVAL;
    std::lock_guard<std::mutex> lock(g_variant_mu);
    const auto key = std::make_tuple(width, height, S);
    if (variant == 0) {
        g_variant.erase(key);
        return SLIC_OK;
    }
    if (!assign_variant_supported(variant, width, height, S)) return SLIC_EINVAL;
    g_variant[key] = variant;
    return SLIC_OK;
}

int slic_get_assign_variant(int32_t width, int32_t height, int32_t S, int32_t* variant) {
    if (width < 1 || height < 1 || S < 1 || !variant) return SLIC_EINVAL;
    *variant = resolve_variant(width, height, S);
    return SLIC_OK;
}

int slic_autotune(const slic_params* p, const uint8_t* d_rgb, int32_t n_iters, int32_t reps,
                  void* hip_stream, void* d_ws, size_t ws_bytes, int32_t* best_variant,
                  float* best_ms_per_iter) {
    if (!params_ok(p) || !d_rgb || !d_ws || !aligned(d_ws) || n_iters < 1 || reps < 1)
        return SLIC_EINVAL;
    if (ws_bytes < slic_workspace_bytes(p)) return SLIC_EINVAL;
    int rc = check_buffers(d_rgb, d_ws);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SLIC_EHIP;
    slic_ctx c;
    bind(&c, p, d_ws, hip_stream);
    int best = 0;
    float best_ms = 0.0f;
    rc = SLIC_OK;
    for (int v = 1; v <= assign_variant_count() && rc == SLIC_OK; ++v) {
        if (!assign_variant_supported(v, p->width, p->height, c.g.S)) continue;
        c.variant = v;
        float total = 0.0f;
        for (int r = 0; r <= reps; ++r) {  // the first round warms up
            c.state = 0;
            if (enqueue_init(&c, d_rgb) != hipSuccess ||
                hipEventRecord(e0, c.stream) != hipSuccess ||
                enqueue_iterations(&c, n_iters) != hipSuccess ||
                hipEventRecord(e1, c.stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = SLIC_EHIP;
                break;
            }
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = SLIC_EHIP;
                break;
            }
            if (r > 0) total += ms;
        }
        const float per_iter = total / static_cast<float>(reps * n_iters);
        if (rc == SLIC_OK && (best == 0 || per_iter < best_ms)) {
            best = v;
            best_ms = per_iter;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SLIC_OK) return rc;
    {
        std::lock_guard<std::mutex> lock(g_variant_mu);
        g_variant[std::make_tuple(p->width, p->height, c.g.S)] = best;
    }
    if (best_variant) *best_variant = best;
    if (best_ms_per_iter) *best_ms_per_iter = best_ms;
    return SLIC_OK;
}

const char* slic_strerror(int code) {
    switch (code) {
        case SLIC_OK: return "ok";
        case SLIC_EINVAL: return "invalid argument";
        case SLIC_ENOMEM: return "out of host memory";
        case SLIC_EHIP: return "HIP runtime error";
        case SLIC_ESTATE: return "invalid context state";
        default: return "unknown error";
    }
}

size_t slic_batch_workspace_bytes(const slic_params* per_image, int32_t n_images) {
    if (!per_image || n_images < 1) return 0;
    for (int i = 0; i < n_images; ++i)
        if (!params_ok(per_image + i)) return 0;
    return batch_layout(per_image, n_images, nullptr, nullptr);
}

int slic_batch_create(slic_batch** out, const slic_params* per_image, int32_t n_images,
                      const uint8_t* const* d_rgb, int32_t* const* d_labels, int32_t n_iters,
                      int32_t enforce, int32_t* d_n_segments, int32_t variant, int32_t use_graph,
                      void* d_ws, size_t ws_bytes) {
    if (!out || !per_image || n_images < 1 || !d_rgb || !d_labels || n_iters < 0 || !d_ws ||
        !aligned(d_ws))
        return SLIC_EINVAL;
    *out = nullptr;
    const size_t need = slic_batch_workspace_bytes(per_image, n_images);
    if (need == 0 || ws_bytes < need) return SLIC_EINVAL;
    for (int i = 0; i < n_images; ++i) {
        if (!d_rgb[i] || !d_labels[i]) return SLIC_EINVAL;
        // one association kernel serves the whole batch: one distance form
        if ((per_image[i].flags & SLIC_DISTANCE_SQUARED) != (per_image[0].flags & SLIC_DISTANCE_SQUARED))
            return SLIC_EINVAL;
    }
    int rc = check_device_ptr(d_ws);
    for (int i = 0; rc == SLIC_OK && i < n_images; ++i) {
        rc = check_device_ptr(d_rgb[i]);
        if (rc == SLIC_OK) rc = check_device_ptr(d_labels[i]);
    }
    if (rc == SLIC_OK && d_n_segments) rc = check_device_ptr(d_n_segments);
    if (rc) return rc;
    slic_batch* b = new (std::nothrow) slic_batch;
    if (!b) return SLIC_ENOMEM;
    b->n = n_images;
    b->params.assign(per_image, per_image + n_images);
    b->rgb.assign(d_rgb, d_rgb + n_images);
    b->labels.assign(d_labels, d_labels + n_images);
    b->n_segments = d_n_segments;
    b->n_iters = n_iters;
    b->enforce = enforce ? 1 : 0;
    b->use_graph = use_graph ? 1 : 0;
    batch_layout(per_image, n_images, b, static_cast<char*>(d_ws));
    b->min_S = b->grids[0].S;
    for (int i = 0; i < n_images; ++i) {
        b->min_S = std::min(b->min_S, b->grids[i].S);
        b->ws[i].labels = b->labels[i];  // associate straight into the caller's buffers
    }
    if (variant != 0 && !batch_variant_ok(b, variant)) {
        delete b;
        return SLIC_EINVAL;
    }
    if (variant == 0) {  // largest tiles every image supports
        int best_area = 0;
        for (int v = 1; v <= assign_variant_count(); ++v) {
            int tw = 0, th = 0;
            assign_variant_shape(v, nullptr, nullptr, &tw, &th);
            if (batch_variant_ok(b, v) && tw * th >= best_area) {
                best_area = tw * th;
                variant = v;
            }
        }
    }
    // the tables are written with synchronous copies: first let every kernel
    // still pending on the device (on any stream, e.g. the last user of this
    // memory) finish
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = batch_upload_lab(b);
    if (e == hipSuccess) e = batch_upload_assign(b, variant);
    if (e == hipSuccess) e = batch_upload_ccl(b);
    if (e == hipSuccess && b->use_graph) e = batch_capture(b);
    if (e != hipSuccess) {
        batch_drop_graph(b);
        delete b;
        return SLIC_EHIP;
    }
    *out = b;
    return SLIC_OK;
}

int slic_batch_run(slic_batch* b, void* hip_stream) {
    if (!b) return SLIC_EINVAL;
    if (b->state != 0) return SLIC_ESTATE;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const hipError_t e = b->exec ? hipGraphLaunch(b->exec, s) : batch_enqueue(b, s);
    if (e != hipSuccess) {
        b->state = 2;
        return SLIC_EHIP;
    }
    return SLIC_OK;
}

int slic_batch_autotune(slic_batch* b, void* hip_stream, int32_t reps, int32_t* best_variant,
                        float* best_ms) {
    if (!b || reps < 1) return SLIC_EINVAL;
    if (b->state != 0) return SLIC_ESTATE;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SLIC_EHIP;
    int best = 0;
    float best_t = 0.0f;
    hipError_t e = hipDeviceSynchronize();  // the tables are rewritten synchronously
    for (int v = 1; e == hipSuccess && v <= assign_variant_count(); ++v) {
        if (!batch_variant_ok(b, v)) continue;
        e = batch_upload_assign(b, v);
        if (e == hipSuccess && b->use_graph) e = batch_capture(b);
        float total = 0.0f;
        for (int r = 0; e == hipSuccess && r <= reps; ++r) {  // the first round warms up
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = b->exec ? hipGraphLaunch(b->exec, s) : batch_enqueue(b, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) total += ms;
        }
        if (e == hipSuccess && (best == 0 || total / reps < best_t)) {
            best = v;
            best_t = total / reps;
        }
    }
    if (e == hipSuccess && best != 0) {
        e = batch_upload_assign(b, best);
        if (e == hipSuccess && b->use_graph) e = batch_capture(b);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        b->state = 2;
        return SLIC_EHIP;
    }
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t;
    return SLIC_OK;
}

void slic_batch_destroy(slic_batch* b) {
    if (!b) return;
    batch_drop_graph(b);
    delete b;
}

int slic_segment_batch(const slic_params* per_image, const uint8_t* const* d_rgb, int32_t n_images,
                       int32_t n_iters, int32_t enforce, int32_t* const* d_labels,
                       int32_t* d_n_segments, void* hip_stream, void* d_ws, size_t ws_bytes) {
    slic_batch* b = nullptr;
    int rc = slic_batch_create(&b, per_image, n_images, d_rgb, d_labels, n_iters, enforce,
                               d_n_segments, 0, 0, d_ws, ws_bytes);
    if (rc) return rc;
    rc = slic_batch_run(b, hip_stream);
    slic_batch_destroy(b);
    return rc;
}

int slic_timing_enable(int32_t on) {
    if (on) {
        for (const TimedLaunch& t : g_launches) {
            g_event_pool.push_back(t.start);
            g_event_pool.push_back(t.stop);
        }
        g_launches.clear();
    }
    g_timing = on != 0;
    return SLIC_OK;
}

int slic_timing_read(const char* prefix, double* total_ms, int64_t* launches) {
    double sum = 0.0;
    int64_t cnt = 0;
    const size_t plen = prefix ? std::strlen(prefix) : 0;
    for (const TimedLaunch& t : g_launches) {
        if (prefix && std::strncmp(t.name, prefix, plen) != 0) continue;
        float ms = 0.0f;
        if (hipEventSynchronize(t.stop) != hipSuccess ||
            hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess)
            return SLIC_EHIP;
        sum += ms;
        ++cnt;
    }
    if (total_ms) *total_ms = sum;
    if (launches) *launches = cnt;
    return SLIC_OK;
}

}  // extern "C"
