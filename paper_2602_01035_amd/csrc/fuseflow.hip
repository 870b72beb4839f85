// Host library and kernels of the fusion path (C ABI in include/fuseflow.h).
//
// Launch structure: one kernel per phase of phases.hpp, each over every frame of the call,
// one workgroup per work item.  ff_fuse enqueues the kernels directly; ff_fuse_batch
// replays them from a HIP graph cached per batch shape.
//
// An earlier single persistent launch running all phases with inter-workgroup waits did
// not finish on the device (cause not established); it is not part of this design.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fuseflow.h"
#include "common.hpp"
#include "internal.hpp"
#include "phases.hpp"

using namespace ff;

// ============================================================================ kernels

// One phase per launch, one workgroup per work item.
template <int KIND, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_phase(Ctx C, uint32_t pass) {
    extern __shared__ __align__(16) char smem[];
    const uint32_t item = blockIdx.x;
    switch (KIND) {
        case PH_BACKPROJECT: ph_backproject(C, item, smem); break;
        case PH_TILE_REDUCE: ph_tile_reduce(C, item, smem); break;
        case PH_HIST: ph_hist(C, item, smem); break;
        case PH_SCAN_A: ph_scan_a(C, item, smem); break;
        case PH_SCAN_M: ph_scan_m(C, item, smem); break;
        case PH_SCAN_B: ph_scan_b(C, item, smem); break;
        case PH_KEYS: ph_keys(C, item, smem); break;
        case PH_RADIX_UP: ph_radix_up<ITEMS>(C, pass, item, smem); break;
        case PH_RADIX_SCAN: ph_radix_scan<ITEMS>(C, pass, item, smem); break;
        case PH_RADIX_DOWN: ph_radix_down<ITEMS>(C, pass, item, smem); break;
        case PH_HEAD_COUNT: ph_head_count<ITEMS>(C, item, smem); break;
        case PH_HEAD_SCAN: ph_head_scan<ITEMS>(C, item, smem); break;
        case PH_HEAD_WRITE: ph_head_write<ITEMS>(C, item, smem); break;
        case PH_FINAL: ph_final(C, item, smem); break;
        case PH_CAM_PREP: ph_cam_prep(C, item, smem); break;
        case PH_CONF: ph_conf(C, item, smem); break;
        case PH_CLASS: ph_class(C, item, smem); break;
        default: break;
    }
}

// The per-cell phase, with a candidate list of KV views (3 covers the common K <= 4 and
// keeps at least four waves resident per SIMD, five at its register and LDS use; 7 covers
// K <= 8).
template <int KV, bool LDS_CAMS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(KV <= 3 ? 4 : 3)))
void k_cells(Ctx C) {
    extern __shared__ __align__(16) char smem[];
    ph_cells<KV, LDS_CAMS>(C, blockIdx.x, smem);
}

// Eq. 3 over one depth map, one thread per pixel (the standalone entry point)
__global__ __launch_bounds__(kBlock) void k_conf_map(const float* D, float* out, int W, int H,
                                                     ConfWeights w) {
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (uint64_t)W * (uint64_t)H) return;
    const int y = (int)(idx / (uint64_t)W), x = (int)(idx - (uint64_t)y * (uint64_t)W);
    glob(out)[idx] = conf_eq3(D, W, H, x, y, w);
}

// Eq. 12, first step: every `stride`-th fused point, grid-stride over kEmcBlocks
// workgroups; per workgroup the sum of the per-point means, the number of points seen by
// at least one camera and the sum of their visible-camera counts
__global__ __launch_bounds__(kBlock) void k_emc(const DevCam* cams, int ncams, const float* xyz,
                                                const uint32_t* count, uint32_t capacity,
                                                float c_occ, uint32_t stride, double* part) {
    __shared__ double s_r[3][kBlock];
    const uint32_t n = min(*glob(count), capacity);
    const uint32_t m = (n + stride - 1) / stride;
    double sum = 0.0, pts = 0.0, vis = 0.0;
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < m; j += gridDim.x * kBlock) {
        const uint64_t i = (uint64_t)j * stride;
        const Pt p{glob(xyz)[3 * i], glob(xyz)[3 * i + 1], glob(xyz)[3 * i + 2]};
        double err;
        uint32_t cnt;
        emc_point(cams, ncams, p, c_occ, err, cnt);
        if (cnt) {
            sum += err / (double)cnt;
            pts += 1.0;
            vis += (double)cnt;
        }
    }
    s_r[0][threadIdx.x] = sum;
    s_r[1][threadIdx.x] = pts;
    s_r[2][threadIdx.x] = vis;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; ++k) s_r[k][threadIdx.x] += s_r[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = s_r[threadIdx.x][0];
}

// Eq. 12, second step: fixed-order sum of the partials; out = {E_MC (m), points, mean
// visible cameras per point}
__global__ __launch_bounds__(kBlock) void k_emc_final(const double* part, int nblocks,
                                                      double* out) {
    __shared__ double s_r[3][kBlock];
    double a[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int k = 0; k < 3; ++k) a[k] += part[b * 3 + k];
    for (int k = 0; k < 3; ++k) s_r[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; ++k) s_r[k][threadIdx.x] += s_r[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double pts = s_r[1][0];
        glob(out)[0] = pts > 0.0 ? s_r[0][0] / pts : 0.0;
        glob(out)[1] = pts;
        glob(out)[2] = pts > 0.0 ? s_r[2][0] / pts : 0.0;
    }
}

// Allocation-free E_MC: the camera records and the per-workgroup partial sums live in a
// file-scope device array instead of a context workspace.  The records arrive as kernel
// arguments (no host staging buffer), kNoAllocCamsPerLaunch per launch.
constexpr int kNoAllocMaxCams = 64;
constexpr int kNoAllocCamsPerLaunch = 16;
constexpr size_t kNoAllocCamBytes = ((sizeof(DevCam) * kNoAllocMaxCams + 255) / 256) * 256;
constexpr size_t kNoAllocScratchBytes = kNoAllocCamBytes + (size_t)kEmcBlocks * 3 * sizeof(double);

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

struct EmcCamArgs {
    float R[9], t[3];
    float fx, fy, cx, cy;
    int32_t W, H;
    const float* depth;
};
struct EmcCamChunk {
    EmcCamArgs cam[kNoAllocCamsPerLaunch];
};

// camera records base .. base + n - 1 of the scratch table, one thread per camera
__global__ __launch_bounds__(64) void k_emc_cams(EmcCamChunk chunk, DevCam* dst, int base, int n) {
    const int k = threadIdx.x;
    if (k >= n) return;
    const EmcCamArgs& a = chunk.cam[k];
    DevCam d{};
    for (int i = 0; i < 9; ++i) d.R[i] = a.R[i];
    for (int i = 0; i < 3; ++i) d.t[i] = a.t[i];
    d.fx = a.fx; d.fy = a.fy; d.cx = a.cx; d.cy = a.cy;
    d.W = a.W; d.H = a.H;
    d.depth = a.depth;
    dst[base + k] = d;
}

// ============================================================================ host side

namespace {

constexpr int kStageSlots = 4;

int ilog2(uint32_t v) {
    int r = 0;
    while ((1u << r) < v) ++r;
    return r;
}

// scatter staging: keys (u64 worst case) and ids of a tile, per-wave and per-tile digit
// counters for the configured digit width, the cameras' pixel offsets
size_t down_smem(int items, int bits, uint32_t ncams, bool key64 = true) {
    const size_t kt = (size_t)kBlock * items;
    return kt * (key64 ? 8 : 4) + kt * 4 + (4 + 2) * ((size_t)1 << bits) * 4 + 32 +
           (size_t)ncams * 4;
}
size_t cells_smem(uint32_t ncams, uint32_t nframes) {
    return cells_layout(ncams, ncams <= (uint32_t)kLdsCams, nframes).total;
}
size_t smem_for(uint32_t kind, int items, uint32_t ncams, int bits, uint32_t nframes,
                bool key64) {
    switch (kind) {
        case PH_BACKPROJECT: return 4 * 8 * 4;
        case PH_TILE_REDUCE: return (8 + 32) * 4;
        case PH_HIST: return kHashSlots * 8;
        case PH_RADIX_UP: return ((size_t)1 << bits) * 4;
        case PH_RADIX_SCAN: return 16 * 4;
        case PH_RADIX_DOWN: return down_smem(items, bits, ncams, key64);
        case PH_HEAD_WRITE: return kMaxFrames * 8 + 16;
        case PH_CELLS: return cells_smem(ncams, nframes);
        case PH_FINAL: return 16;
        default: return 64;
    }
}

}  // namespace

struct ff_context {
    int device = 0;
    uint64_t max_pixels = 0;
    int32_t max_cams = 0, max_frames = 0;
    // descriptors
    size_t desc_bytes = 0;
    char* d_desc = nullptr;
    char* h_stage[kStageSlots] = {};
    hipEvent_t stage_ev[kStageSlots] = {};
    int stage = 0;
    // workspace
    BatchState* bs = nullptr;
    FrameState* fs = nullptr;
    TilePart* tiles = nullptr;
    uint32_t* tile_off = nullptr;
    uint32_t* counts = nullptr;
    uint64_t* fine_base = nullptr;
    uint64_t counts_cap = 0;
    uint8_t* level = nullptr;
    CamClass* cls = nullptr;
    uint64_t* scan_tile = nullptr;
    void* keysA = nullptr;
    void* keysB = nullptr;
    uint32_t* valsA = nullptr;
    uint32_t* valsB = nullptr;
    uint32_t* digit_hist = nullptr;
    uint32_t* digit_total = nullptr;
    uint32_t* head_cnt = nullptr;
    uint32_t* cell_start = nullptr;
    uint32_t* conf_sorted = nullptr;
    CamLite* camlite = nullptr;
    float* raytab = nullptr;
    uint64_t raytab_cap = 0;
    float* conf_ws = nullptr;          // Eq. 3 confidence of every pixel (FF_CONF_EQ3)
    double* emc_part = nullptr;        // per-workgroup partial sums of the E_MC evaluator
    uint64_t sort_tiles_cap = 0;
    hipEvent_t last = nullptr;
    bool have_last = false;
    std::vector<void*> allocs;
    ff_tuning tune{8, 8, 0, 0, 1};                // default tuning
    std::map<std::string, ff_tuning> tuned;       // tuning per batch shape
    std::string device_name;
    int n_cu = 0;                                 // compute units of the device
    std::map<uint64_t, uint32_t> cells_fit;       // resident per-cell workgroups by launch shape
    hipStream_t cap_stream = nullptr;
    std::map<std::string, hipGraphExec_t> graphs;
    // kernel tracing (events on the call's stream)
    bool trace = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;
    std::vector<int> tslot;
    size_t tused = 0;
    ff_trace tacc{};
    // timing of one kernel inside every call, graph replays included (events on the
    // call's stream just before and after that kernel)
    int32_t probe_slot = -1;
    struct ProbeRec {
        hipEvent_t a, b;
        uint32_t frames;
        uint64_t pixels;
    };
    std::vector<ProbeRec> probe_pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> probe_free;
    ff_probe pacc{};
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

#define FF_HIP(call)                                    \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) {                         \
            (void)hipGetLastError();                    \
            return FF_ERR_HIP;                          \
        }                                               \
    } while (0)

ff_status dalloc(ff_context* c, void** p, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return FF_ERR_OOM;
    }
    c->allocs.push_back(*p);
    return FF_OK;
}

// All sizes that depend only on the context limits.
// descriptor: header, frames, cameras, then the camera of every pixel tile (u16)
size_t tile_cam_offset(int32_t F, int32_t C) {
    return (sizeof(CallHdr) + sizeof(DevFrame) * (size_t)F + sizeof(DevCam) * (size_t)C + 15) &
           ~(size_t)15;
}

struct Sizes {
    uint64_t desc, counts, scan, keys, px_tiles, sort_tiles, cell, dhist;
};
Sizes sizes_for(uint64_t P, int32_t C, int32_t F) {
    Sizes s;
    s.px_tiles = P / kPxTile + (uint64_t)C + 1;
    s.desc = tile_cam_offset(F, C) + 2 * s.px_tiles;
    s.counts = (uint64_t)F * 64 * 64 * 64;           // grows on demand for coarse_res > 64
    s.scan = (s.counts + kScanTile - 1) / kScanTile + 1;
    s.keys = P + 1;
    s.sort_tiles = P / (kBlock * 8) + 2;              // sort tiles hold >= 8 keys per thread
    s.cell = P + 2;
    s.dhist = (uint64_t)kMaxDigits * s.sort_tiles;
    return s;
}

// Camera parameters for which the per-cell kernel's approximate field-of-view pre-test is
// proven to take the exact decisions: all finite, image sides and principal point within
// 2^14 px, focal lengths 2^-20 <= |f| <= 2^20 px.
bool camera_ok(const ff_camera& cm) {
    if (cm.width < 1 || cm.height < 1 || cm.width > 16384 || cm.height > 16384) return false;
    for (float f : {cm.fx, cm.fy})
        if (!std::isfinite(f) || !(std::fabs(f) >= 0x1p-20f && std::fabs(f) <= 0x1p20f))
            return false;
    for (float c : {cm.cx, cm.cy})
        if (!std::isfinite(c) || std::fabs(c) > 16384.0f) return false;
    for (float v : cm.world_to_cam)
        if (!std::isfinite(v)) return false;
    return true;
}

ff_status validate_params(const ff_params* p) {
    if (!p) return FF_ERR_INVALID_ARG;
    const int G = p->coarse_res;
    if (G < 1 || G > 128 || (G & (G - 1))) return FF_ERR_INVALID_ARG;
    if (p->max_level < 0 || p->max_level > 16) return FF_ERR_INVALID_ARG;
    if (3 * (ilog2((uint32_t)G) + p->max_level) > 56) return FF_ERR_INVALID_ARG;
    if (p->level_override < -1 || p->level_override > p->max_level) return FF_ERR_INVALID_ARG;
    if (p->target_per_cell < 1 || p->k_views < 1 || p->k_views > kMaxK) return FF_ERR_INVALID_ARG;
    if (!(p->sigma > 0.0f) || !std::isfinite(p->sigma)) return FF_ERR_INVALID_ARG;
    if (!std::isfinite(p->tau)) return FF_ERR_INVALID_ARG;
    if (p->flags & ~15u) return FF_ERR_INVALID_ARG;
    return FF_OK;
}

}  // namespace

ff_status ff::check_frame(const ff_frame& fr, const ff_params& prm, const ff_output& o) {
    if (validate_params(&prm) != FF_OK) return FF_ERR_INVALID_ARG;
    if (fr.n_cams < 1 || fr.n_cams > kMaxCamsPerFrame || !fr.cams || !fr.views)
        return FF_ERR_INVALID_ARG;
    if (!o.xyz || !o.weight || !o.count || !o.status) return FF_ERR_INVALID_ARG;
    if (o.member_ids && !o.member_offsets) return FF_ERR_INVALID_ARG;
    const bool conf_eq3 = (prm.flags & FF_CONF_EQ3) != 0;
    uint64_t P = 0;
    bool all_rgb = true;
    for (int32_t k = 0; k < fr.n_cams; ++k) {
        const ff_camera& cm = fr.cams[k];
        const ff_view& v = fr.views[k];
        if (!camera_ok(cm) || !v.depth || (!v.conf && !conf_eq3)) return FF_ERR_INVALID_ARG;
        P += (uint64_t)cm.width * (uint64_t)cm.height;
        all_rgb = all_rgb && v.rgb;
    }
    if (P >= 0xFFFFFFFFull || (o.rgb && !all_rgb)) return FF_ERR_INVALID_ARG;
    return FF_OK;
}

namespace {

void drop_graphs(ff_context* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

ff_status grow_counts(ff_context* c, uint64_t need, hipStream_t stream) {
    if (need <= c->counts_cap) return FF_OK;
    // rare: a larger coarse grid than the workspace was sized for; wait, then regrow
    FF_HIP(hipStreamSynchronize(stream));
    if (c->have_last) FF_HIP(hipEventSynchronize(c->last));
    auto drop = [&](void* p) {
        (void)hipFree(p);
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), p), c->allocs.end());
    };
    drop(c->counts);
    drop(c->fine_base);
    drop(c->level);
    drop(c->cls);
    drop(c->scan_tile);
    c->counts = nullptr; c->fine_base = nullptr; c->level = nullptr; c->cls = nullptr;
    c->scan_tile = nullptr;
    ff_status st;
    if ((st = dalloc(c, (void**)&c->counts, need * 4 * kCountStripes)) != FF_OK) return st;
    if ((st = dalloc(c, (void**)&c->fine_base, need * 8)) != FF_OK) return st;
    if ((st = dalloc(c, (void**)&c->level, need)) != FF_OK) return st;
    if ((st = dalloc(c, (void**)&c->cls, need * sizeof(CamClass))) != FF_OK) return st;
    if ((st = dalloc(c, (void**)&c->scan_tile, ((need + kScanTile - 1) / kScanTile + 1) * 8)) != FF_OK)
        return st;
    c->counts_cap = need;
    drop_graphs(c);      // the captured kernels hold the old pointers
    return FF_OK;
}

// The key of a batch shape in the tuning cache: every frame's camera resolutions in order,
// the grid and level limits, the flags and the view-list size.  Empty when the batch is not
// well formed (the call itself then reports the error).
std::string shape_key(int32_t n_frames, const ff_frame* frames, const ff_params* prm) {
    std::string k;
    if (n_frames < 1 || !frames || !prm) return k;
    char buf[96];
    for (int32_t f = 0; f < n_frames; ++f) {
        if (frames[f].n_cams < 1 || !frames[f].cams) return std::string();
        for (int32_t i = 0; i < frames[f].n_cams; ++i) {
            std::snprintf(buf, sizeof(buf), "%dx%d,", frames[f].cams[i].width, frames[f].cams[i].height);
            k += buf;
        }
        k += ";";
    }
    std::snprintf(buf, sizeof(buf), "|G%d|L%d|f%u|w%d", prm->coarse_res, prm->max_level,
                  prm->flags, prm->k_views > 4 ? 1 : 0);
    return k + buf;
}

bool tuning_ok(const ff_tuning& t) {
    return t.radix_bits >= 6 && t.radix_bits <= kMaxRadixBits &&
           (t.sort_items == 8 || t.sort_items == 16) && t.hist_tiles >= 0 &&
           t.hist_tiles <= kMaxHistTiles && (t.cell_groups == 0 ||
           (t.cell_groups >= 64 && t.cell_groups <= 4096)) &&
           (t.use_graph == 0 || t.use_graph == 1);
}

const ff_tuning& tuning_for(const ff_context* c, const std::string& key) {
    auto it = c->tuned.find(key);
    return it == c->tuned.end() ? c->tune : it->second;
}

Ctx make_ctx(ff_context* c) {
    Ctx C;
    C.hdr = reinterpret_cast<const CallHdr*>(c->d_desc);
    C.frames = reinterpret_cast<const DevFrame*>(c->d_desc + sizeof(CallHdr));
    C.cams = reinterpret_cast<DevCam*>(c->d_desc + sizeof(CallHdr) +
                                       sizeof(DevFrame) * (size_t)c->max_frames);
    C.tile_cam = reinterpret_cast<const uint16_t*>(c->d_desc +
                                                   tile_cam_offset(c->max_frames, c->max_cams));
    C.bs = c->bs;
    C.fs = c->fs;
    C.tiles = c->tiles;
    C.tile_off = c->tile_off;
    C.counts = c->counts;
    C.fine_base = c->fine_base;
    C.level = c->level;
    C.cls = c->cls;
    C.scan_tile = c->scan_tile;
    C.keysA = c->keysA;
    C.keysB = c->keysB;
    C.valsA = c->valsA;
    C.valsB = c->valsB;
    C.digit_hist = c->digit_hist;
    C.digit_total = c->digit_total;
    C.head_cnt = c->head_cnt;
    C.cell_start = c->cell_start;
    C.conf_sorted = c->conf_sorted;
    C.camlite = c->camlite;
    C.raytab = c->raytab;
    C.P_cap = (uint32_t)std::min<uint64_t>(c->max_pixels, 0xFFFFFFFEull);
    C.sort_tiles_cap = (uint32_t)c->sort_tiles_cap;
    return C;
}

struct Launch {
    uint32_t kind, n, pass;
};
struct Plan {
    std::vector<Launch> launches;
    int sort_items = 8;         // keys per thread of the sort tiles
    uint32_t ncams = 0;
    bool wide_views = false;    // K - 1 > 3 kept views
    size_t desc_used = 0;       // bytes of the descriptor this call fills
    int radix_bits = 10;        // widest digit of the sort passes
    uint32_t nframes = 0;
    bool key64_ok = true;       // the key-width bound allows 64-bit keys (scatter LDS size)
};

// Validate one batch and fill the host staging descriptor.  Returns the launch plan and a
// key describing everything the plan depends on (for the graph cache).
// Workgroups of the per-cell kernel that the whole device holds at once for a launch shape
// (kernel variant and LDS bytes): how many share a CU follows from their registers and LDS.
uint32_t cells_resident(ff_context* c, bool wide, bool lds, size_t smem) {
    const uint64_t key = ((uint64_t)(wide ? 2u : 0u) | (lds ? 1u : 0u)) << 32 | (uint64_t)smem;
    const auto it = c->cells_fit.find(key);
    if (it != c->cells_fit.end()) return it->second;
    const void* f = wide ? (lds ? (const void*)k_cells<kMaxK - 1, true>
                                : (const void*)k_cells<kMaxK - 1, false>)
                         : (lds ? (const void*)k_cells<3, true> : (const void*)k_cells<3, false>);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlock, smem) != hipSuccess ||
        per_cu < 1)
        per_cu = 4;
    const uint32_t r = (uint32_t)std::max(1, c->n_cu > 0 ? c->n_cu : 256) * (uint32_t)per_cu;
    c->cells_fit[key] = r;
    return r;
}

ff_status build_desc(ff_context* c, int32_t n_frames, const ff_frame* frames,
                     const ff_params* prm, const ff_output* outs, const ff_tuning& T,
                     char* stage, Plan& plan, std::string& shape) {
    if (n_frames < 1 || n_frames > c->max_frames || !frames || !outs) return FF_ERR_INVALID_ARG;
    ff_status st = validate_params(prm);
    if (st != FF_OK) return st;
    CallHdr* H = reinterpret_cast<CallHdr*>(stage);
    DevFrame* F = reinterpret_cast<DevFrame*>(stage + sizeof(CallHdr));
    DevCam* K = reinterpret_cast<DevCam*>(stage + sizeof(CallHdr) +
                                          sizeof(DevFrame) * (size_t)c->max_frames);
    const size_t tc_off = tile_cam_offset(c->max_frames, c->max_cams);
    uint16_t* TC = reinterpret_cast<uint16_t*>(stage + tc_off);
    const uint64_t tc_cap = (c->desc_bytes - tc_off) / 2;
    std::memset(H, 0, sizeof(CallHdr));
    uint64_t P = 0, tab = 0;
    uint32_t ncam = 0, ntile = 0;
    const bool conf_eq3 = (prm->flags & FF_CONF_EQ3) != 0;
    char buf[64];
    for (int32_t f = 0; f < n_frames; ++f) {
        const ff_frame& fr = frames[f];
        const ff_output& o = outs[f];
        if (fr.n_cams < 1 || fr.n_cams > kMaxCamsPerFrame || !fr.cams || !fr.views)
            return FF_ERR_INVALID_ARG;
        if ((int64_t)ncam + fr.n_cams > c->max_cams) return FF_ERR_INVALID_ARG;
        if (!o.xyz || !o.weight || !o.count || !o.status) return FF_ERR_INVALID_ARG;
        if (o.member_ids && !o.member_offsets) return FF_ERR_INVALID_ARG;
        DevFrame& df = F[f];
        std::memset(&df, 0, sizeof(DevFrame));
        df.cam_begin = ncam;
        df.n_cams = (uint32_t)fr.n_cams;
        df.pix_begin = (uint32_t)P;
        df.tile_begin = ntile;
        bool all_rgb = true;
        uint64_t fpix = 0;
        for (int32_t k = 0; k < fr.n_cams; ++k) {
            const ff_camera& cm = fr.cams[k];
            const ff_view& v = fr.views[k];
            if (!camera_ok(cm) || !v.depth || (!v.conf && !conf_eq3)) return FF_ERR_INVALID_ARG;
            const uint64_t npx = (uint64_t)cm.width * (uint64_t)cm.height;
            DevCam& d = K[ncam];
            std::memset(&d, 0, sizeof(DevCam));
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) d.R[i * 3 + j] = cm.world_to_cam[i * 4 + j];
                d.t[i] = cm.world_to_cam[i * 4 + 3];
            }
            d.fx = cm.fx; d.fy = cm.fy; d.cx = cm.cx; d.cy = cm.cy;
            d.W = cm.width; d.H = cm.height;
            d.pix_off = (uint32_t)P;
            d.frame_pix_off = (uint32_t)fpix;
            d.tile_off = ntile;
            d.frame = (uint32_t)f;
            // with FF_CONF_EQ3 the confidence is computed into the workspace first
            const float* conf = conf_eq3 ? c->conf_ws + P : v.conf;
            d.conf_out = conf_eq3 ? c->conf_ws + P : nullptr;
            d.vec_ok = ((uintptr_t)v.depth % 16 == 0 && (uintptr_t)conf % 16 == 0) ? 1u : 0u;
            d.tab_off = (uint32_t)tab;
            tab += (uint64_t)cm.width + (uint64_t)cm.height;
            if (tab > c->raytab_cap) return FF_ERR_INVALID_ARG;
            d.depth = v.depth;
            d.conf = conf;
            d.rgb = v.rgb;
            all_rgb = all_rgb && v.rgb;
            const uint64_t nt = (npx + kPxTile - 1) / kPxTile;
            if (ntile + nt > tc_cap) return FF_ERR_INVALID_ARG;    // more pixels than sized for
            for (uint64_t t = 0; t < nt; ++t) TC[ntile + t] = (uint16_t)ncam;
            ntile += (uint32_t)nt;
            P += npx;
            fpix += npx;
            ++ncam;
            if (P >= 0xFFFFFFFFull || P > c->max_pixels) return FF_ERR_INVALID_ARG;
            std::snprintf(buf, sizeof(buf), "%dx%d,", cm.width, cm.height);
            shape += buf;
        }
        if (o.rgb && !all_rgb) return FF_ERR_INVALID_ARG;
        shape += ";";
        df.n_pix = (uint32_t)fpix;
        df.n_tiles = ntile - df.tile_begin;
        df.has_rgb = all_rgb ? 1u : 0u;
        df.xyz = o.xyz; df.weight = o.weight; df.rgb = o.rgb;
        df.n_members = o.n_members; df.reps = o.reps; df.keys = o.keys;
        df.moff = o.member_offsets; df.mids = o.member_ids;
        if (o.member_ids) H->any_mids = 1;
        df.capacity = o.capacity; df.member_capacity = o.member_capacity;
        df.count = o.count; df.status = o.status; df.info = o.info;
    }
    const int G = prm->coarse_res;
    const uint64_t G3 = (uint64_t)G * G * G;
    H->prm.tau = prm->tau;
    H->prm.K = prm->k_views;
    H->prm.sigma = prm->sigma;
    H->prm.G = G;
    H->prm.log2G = ilog2((uint32_t)G);
    H->prm.Lmax = prm->max_level;
    H->prm.target = prm->target_per_cell;
    H->prm.level_override = prm->level_override;
    H->prm.flags = prm->flags;
    H->n_frames = (uint32_t)n_frames;
    H->n_cams = ncam;
    H->lds_cams = ncam <= (uint32_t)kLdsCams ? 1u : 0u;
    plan.ncams = ncam;
    plan.nframes = (uint32_t)n_frames;
    plan.wide_views = prm->k_views > 4;
    plan.radix_bits = T.radix_bits;
    plan.sort_items = T.sort_items;
    H->n_px_tiles = ntile;
    plan.desc_used = tc_off + 2 * (size_t)ntile;
    H->P_tot = (uint32_t)P;
    const bool no_sa = prm->flags & FF_NO_SA;
    const uint64_t ncounts = no_sa ? 0 : (uint64_t)n_frames * G3;
    H->n_counts = (uint32_t)ncounts;
    H->n_scan_tiles = (uint32_t)std::max<uint64_t>(1, (ncounts + kScanTile - 1) / kScanTile);
    const uint32_t KT = (uint32_t)(kBlock * T.sort_items);
    H->sort_items = (uint32_t)T.sort_items;
    // histogram tiles per workgroup: about 900 workgroups (3.5 per CU) measured fastest,
    // from one 1280x720 camera (225 tiles: 1 each) to two 16-camera frames (8 each)
    H->hist_tiles = T.hist_tiles > 0
                        ? (uint32_t)T.hist_tiles
                        : (uint32_t)std::min<uint64_t>(kMaxHistTiles,
                                                       std::max<uint64_t>(1, (ntile + 450) / 900));
    H->n_sort_tiles = (uint32_t)std::max<uint64_t>(1, (P + KT - 1) / KT);
    // per-cell phase: waves walk 64-cell steps.  Up to one 8x1280x720 frame: the workgroups
    // that fit resident at once (5 per CU at its register and LDS use, 1280), so no partial
    // second round trails the launch, and small frames still spread over every CU; larger
    // batches: two full rounds, which balance their uneven cells better (measured at two
    // such frames: 2560 workgroups 130 us per frame, 2048 140, 1280 137)
    {
        const uint32_t resident = cells_resident(c, plan.wide_views, ncam <= (uint32_t)kLdsCams,
                                                 cells_smem(ncam, (uint32_t)n_frames));
        H->n_cell_items = T.cell_groups > 0 ? (uint32_t)T.cell_groups
                          : P <= 7372800ull ? resident : 2u * resident;
    }
    H->max_radix_bits = (uint32_t)T.radix_bits;
    // Widest possible dense key.  The key range T is the sum over occupied coarse cells of
    // 8^L.  A cell refined to level L >= 1 holds more than target 4^(L-1) points (level L-1
    // did not suffice), so it spends fewer than 2^(L+2) / target key values per point; a
    // level-0 cell spends at most one.  Hence T <= M max(1, 2^(Lmax+2) / target) with M <= P
    // points; a forced level L gives T <= min(M, cells) 8^L; and always T <= cells 8^Lmax.
    {
        const uint64_t cells = (uint64_t)n_frames * G3;
        const int lo = prm->level_override;
        const uint64_t cap = cells << (3 * prm->max_level);
        uint64_t bound;
        if (lo >= 0) {
            bound = std::min<uint64_t>(P, cells) << (3 * lo);
        } else {
            const uint64_t per = std::max<uint64_t>(
                1, ((1ull << (prm->max_level + 2)) + (uint64_t)prm->target_per_cell - 1) /
                       (uint64_t)prm->target_per_cell);
            bound = (P > cap / per) ? cap : std::min<uint64_t>(cap, P * per);
        }
        const uint32_t bits_max = bound > 1 ? (uint32_t)(64 - __builtin_clzll(bound - 1)) : 0u;
        H->npass_max = std::max<uint32_t>(1, (bits_max + H->max_radix_bits - 1) / H->max_radix_bits);
        // keys stay 32-bit on the device whenever the bound allows no more: the scatter
        // then stages 4-byte keys and more of its workgroups fit per CU
        H->key64_ok = bits_max > 32 ? 1u : 0u;
        plan.key64_ok = bits_max > 32;
    }
    if (H->npass_max > (uint32_t)kMaxPass) return FF_ERR_INVALID_ARG;
    plan.launches.clear();
    auto add = [&](uint32_t kind, uint32_t n, uint32_t pass) { plan.launches.push_back({kind, n, pass}); };
    if (conf_eq3) add(PH_CONF, ntile, 0);
    add(PH_CAM_PREP, ncam, 0);
    add(PH_BACKPROJECT, ntile, 0);
    add(PH_TILE_REDUCE, (uint32_t)n_frames, 0);
    if (!no_sa) {
        add(PH_HIST, (ntile + H->hist_tiles - 1) / H->hist_tiles, 0);
        add(PH_SCAN_A, H->n_scan_tiles, 0);
        add(PH_SCAN_M, 1, 0);
        add(PH_SCAN_B, H->n_scan_tiles, 0);
        if (!(prm->flags & FF_NO_DC)) {
            // camera slots per coarse cell: a power of two >= the largest frame's cameras
            uint32_t lanes = 0, most = 1;
            for (int32_t f = 0; f < n_frames; ++f) most = std::max<uint32_t>(most, (uint32_t)frames[f].n_cams);
            while ((1u << lanes) < most) ++lanes;
            H->cls_lanes = lanes;
            add(PH_CLASS, (uint32_t)(((ncounts << lanes) + kBlock - 1) / kBlock), 0);
        }
    }
    add(PH_KEYS, ntile, 0);
    if (!no_sa) {
        const uint32_t D = 1u << H->max_radix_bits;
        for (uint32_t k = 0; k < H->npass_max; ++k) {
            add(PH_RADIX_UP, H->n_sort_tiles, k);
            add(PH_RADIX_SCAN, D, k);
            add(PH_RADIX_DOWN, H->n_sort_tiles, k);
        }
        add(PH_HEAD_COUNT, H->n_sort_tiles, 0);
        add(PH_HEAD_SCAN, 1, 0);
        add(PH_HEAD_WRITE, H->n_sort_tiles, 0);
    }
    add(PH_CELLS, H->n_cell_items, 0);
    add(PH_FINAL, 1, 0);
    char tail[96];
    // everything the captured launches depend on besides the per-camera sizes above: grid
    // and level limits, flags, the per-cell kernel variant, tuning, and the sort's pass
    // count and key width (set by the level limits and the target count through the
    // key-width bound; the key width sizes the scatter's LDS)
    std::snprintf(tail, sizeof(tail), "|G%d|L%d|f%u|w%d|t%d,%d,%d,%d|p%u,%u", G, prm->max_level,
                  prm->flags, plan.wide_views ? 1 : 0, T.radix_bits, T.sort_items,
                  T.hist_tiles, T.cell_groups, H->npass_max, H->key64_ok);
    shape += tail;
    return FF_OK;
}

int trace_slot(const Launch& L) {
    if (L.kind == PH_CONF) return kTraceSlotConf;
    if (L.kind == PH_CLASS) return kTraceSlotClass;
    if (L.kind == PH_RADIX_UP || L.kind == PH_RADIX_SCAN || L.kind == PH_RADIX_DOWN)
        return std::min(30, 16 + 3 * (int)L.pass + (int)(L.kind - PH_RADIX_UP));
    return (int)L.kind;
}

// accumulate the timed launches of the previous call (waits for it)
ff_status trace_collect(ff_context* c) {
    if (c->tused == 0) return FF_OK;
    FF_HIP(hipEventSynchronize(c->tev[c->tused - 1].second));
    for (size_t i = 0; i < c->tused; ++i) {
        float ms = 0;
        FF_HIP(hipEventElapsedTime(&ms, c->tev[i].first, c->tev[i].second));
        c->tacc.total_ms[c->tslot[i]] += ms;
        c->tacc.launches[c->tslot[i]] += 1;
    }
    c->tacc.calls += 1;
    c->tused = 0;
    return FF_OK;
}

ff_status trace_mark(ff_context* c, int slot, bool begin, hipStream_t s) {
    if (begin) {
        if (c->tused == c->tev.size()) {
            hipEvent_t a, b;
            FF_HIP(hipEventCreate(&a));
            FF_HIP(hipEventCreate(&b));
            c->tev.push_back({a, b});
            c->tslot.push_back(0);
        }
        c->tslot[c->tused] = slot;
        FF_HIP(hipEventRecord(c->tev[c->tused].first, s));
    } else {
        FF_HIP(hipEventRecord(c->tev[c->tused].second, s));
        ++c->tused;
    }
    return FF_OK;
}

// harvest finished probe records in call order; `all` waits for every one
ff_status probe_collect(ff_context* c, bool all) {
    size_t done = 0;
    ff_status st = FF_OK;
    for (; done < c->probe_pending.size(); ++done) {
        const ff_context::ProbeRec& r = c->probe_pending[done];
        hipError_t q = all ? hipEventSynchronize(r.b) : hipEventQuery(r.b);
        if (q == hipErrorNotReady) break;
        float ms = 0;
        if (q != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            (void)hipGetLastError();
            st = FF_ERR_HIP;
        } else {
            c->pacc.total_ms += ms;
            c->pacc.launches += 1;
            c->pacc.frames += r.frames;
            c->pacc.pixels += r.pixels;
        }
        c->probe_free.push_back({r.a, r.b});
    }
    c->probe_pending.erase(c->probe_pending.begin(), c->probe_pending.begin() + done);
    return st;
}

ff_status probe_mark(ff_context* c, bool begin, hipStream_t s, uint32_t frames,
                     uint64_t pixels) {
    if (begin) {
        if (c->probe_free.empty()) {
            hipEvent_t a, b;
            FF_HIP(hipEventCreate(&a));
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return FF_ERR_HIP;
            }
            c->probe_free.push_back({a, b});
        }
        const auto ev = c->probe_free.back();
        c->probe_free.pop_back();
        c->probe_pending.push_back({ev.first, ev.second, frames, pixels});
        FF_HIP(hipEventRecord(ev.first, s));
    } else {
        FF_HIP(hipEventRecord(c->probe_pending.back().b, s));
    }
    return FF_OK;
}

void launch_cells(const Ctx& C, uint32_t ncams, const Plan& plan, hipStream_t s, dim3 grid,
                  dim3 block, size_t smem) {
    const bool lds = ncams <= (uint32_t)kLdsCams;
    if (plan.wide_views) {
        if (lds) hipLaunchKernelGGL((k_cells<kMaxK - 1, true>), grid, block, smem, s, C);
        else hipLaunchKernelGGL((k_cells<kMaxK - 1, false>), grid, block, smem, s, C);
    } else {
        if (lds) hipLaunchKernelGGL((k_cells<3, true>), grid, block, smem, s, C);
        else hipLaunchKernelGGL((k_cells<3, false>), grid, block, smem, s, C);
    }
}

template <int ITEMS>
void launch_one(const Ctx& C, const Launch& L, uint32_t ncams, const Plan& plan, hipStream_t s) {
    const size_t smem =
        smem_for(L.kind, ITEMS, ncams, plan.radix_bits, plan.nframes, plan.key64_ok);
    const dim3 grid(std::max<uint32_t>(1, L.n)), block(kBlock);
#define FF_L(K) hipLaunchKernelGGL((k_phase<K, ITEMS>), grid, block, smem, s, C, L.pass)
    switch (L.kind) {
        case PH_BACKPROJECT: FF_L(PH_BACKPROJECT); break;
        case PH_TILE_REDUCE: FF_L(PH_TILE_REDUCE); break;
        case PH_HIST: FF_L(PH_HIST); break;
        case PH_SCAN_A: FF_L(PH_SCAN_A); break;
        case PH_SCAN_M: FF_L(PH_SCAN_M); break;
        case PH_SCAN_B: FF_L(PH_SCAN_B); break;
        case PH_KEYS: FF_L(PH_KEYS); break;
        case PH_RADIX_UP: FF_L(PH_RADIX_UP); break;
        case PH_RADIX_SCAN: FF_L(PH_RADIX_SCAN); break;
        case PH_RADIX_DOWN: FF_L(PH_RADIX_DOWN); break;
        case PH_HEAD_COUNT: FF_L(PH_HEAD_COUNT); break;
        case PH_HEAD_SCAN: FF_L(PH_HEAD_SCAN); break;
        case PH_HEAD_WRITE: FF_L(PH_HEAD_WRITE); break;
        case PH_CELLS: launch_cells(C, ncams, plan, s, grid, block, smem); break;
        case PH_FINAL: FF_L(PH_FINAL); break;
        case PH_CAM_PREP: FF_L(PH_CAM_PREP); break;
        case PH_CONF: FF_L(PH_CONF); break;
        case PH_CLASS: FF_L(PH_CLASS); break;
        default: break;
    }
#undef FF_L
}

template <int ITEMS>
ff_status run_plain(ff_context* c, const Ctx& C, const Plan& plan, hipStream_t s) {
    const bool tr = c->trace;
    for (const Launch& L : plan.launches) {
        if (tr) { ff_status st = trace_mark(c, trace_slot(L), true, s); if (st != FF_OK) return st; }
        launch_one<ITEMS>(C, L, plan.ncams, plan, s);
        if (tr) { ff_status st = trace_mark(c, trace_slot(L), false, s); if (st != FF_OK) return st; }
    }
    FF_HIP(hipGetLastError());
    return FF_OK;
}

ff_status dispatch_plain(ff_context* c, const Ctx& C, const Plan& plan, hipStream_t s) {
    switch (plan.sort_items) {
        case 16: return run_plain<16>(c, C, plan, s);
        default: return run_plain<8>(c, C, plan, s);
    }
}

// Replay the batch's kernels from a graph captured once per shape (resolution mix,
// frame count, grid parameters and tuning): one launch per batch on the stream.
ff_status run_graph(ff_context* c, const Ctx& C, const Plan& plan, const std::string& key,
                    hipStream_t s) {
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        FF_HIP(hipGraphLaunch(it->second, s));
        return FF_OK;
    }
    // the first batch of a shape: its kernels go to the stream at once, and the graph for
    // the next ones is captured (on a stream of its own) and instantiated while they run
    if (c->graphs.size() >= 64) {
        FF_HIP(hipStreamSynchronize(s));
        drop_graphs(c);
    }
    ff_status st = dispatch_plain(c, C, plan, s);
    if (st != FF_OK) return st;
    hipGraph_t g = nullptr;
    FF_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    st = dispatch_plain(c, C, plan, c->cap_stream);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != FF_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    FF_HIP(e);
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FF_HIP(e);
    c->graphs.emplace(key, ex);
    return FF_OK;
}

// The plan with the probed kernel launched on its own between events; the launches
// around it run as before (replayed from graphs cached per segment, or enqueued).
ff_status run_probed(ff_context* c, const Ctx& C, const Plan& plan, const std::string& shape,
                     hipStream_t s, bool graph, uint32_t frames, uint64_t pixels) {
    Plan seg = plan;            // every launch parameter of the plan, segment by segment
    seg.launches.clear();
    int nseg = 0;
    auto flush = [&]() -> ff_status {
        if (seg.launches.empty()) return FF_OK;
        ff_status st = graph ? run_graph(c, C, seg,
                                         shape + "|seg" + std::to_string(nseg) + "|probe" +
                                             std::to_string(c->probe_slot),
                                         s)
                             : dispatch_plain(c, C, seg, s);
        ++nseg;
        seg.launches.clear();
        return st;
    };
    for (const Launch& L : plan.launches) {
        if (trace_slot(L) != c->probe_slot) {
            seg.launches.push_back(L);
            continue;
        }
        ff_status st = flush();
        if (st != FF_OK) return st;
        if ((st = probe_mark(c, true, s, frames, pixels)) != FF_OK) return st;
        seg.launches.push_back(L);
        st = dispatch_plain(c, C, seg, s);
        seg.launches.clear();
        if (st != FF_OK) return st;
        if ((st = probe_mark(c, false, s, frames, pixels)) != FF_OK) return st;
    }
    return flush();
}

ff_status set_smem_limits() {
    static std::once_flag once;
    static ff_status result = FF_OK;
    std::call_once(once, [] {
        auto setk = [](const void* f, size_t b) {
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b) != hipSuccess)
                result = FF_ERR_HIP;
        };
        setk((const void*)k_phase<PH_RADIX_DOWN, 8>, down_smem(8, 10, kMaxBatchCams));
        setk((const void*)k_phase<PH_RADIX_DOWN, 16>, down_smem(16, 10, kMaxBatchCams));
        const size_t cs = std::max(cells_smem((uint32_t)kLdsCams, (uint32_t)kMaxFrames),
                                   cells_smem((uint32_t)kMaxBatchCams, (uint32_t)kMaxFrames));
        setk((const void*)k_cells<3, true>, cs);
        setk((const void*)k_cells<3, false>, cs);
        setk((const void*)k_cells<kMaxK - 1, true>, cs);
        setk((const void*)k_cells<kMaxK - 1, false>, cs);
    });
    return result;
}

}  // namespace

// ============================================================================ C ABI

extern "C" {

const char* ff_version(void) { return "fuseflow-mi355x 0.2 (gfx950)"; }

const char* ff_status_string(ff_status s) {
    switch (s) {
        case FF_OK: return "ok";
        case FF_ERR_INVALID_ARG: return "invalid argument";
        case FF_ERR_OOM: return "out of memory";
        case FF_ERR_BUSY: return "busy";
        case FF_ERR_HIP: return "HIP runtime error";
        case FF_ERR_NOT_FOUND: return "not found";
    }
    return "unknown status";
}

void ff_params_default(ff_params* p) {
    if (!p) return;
    p->tau = 0.6f;
    p->k_views = 4;
    p->sigma = 0.02f;
    p->coarse_res = 64;
    p->max_level = 6;
    p->target_per_cell = 16;
    p->level_override = -1;
    p->flags = 0;
}

uint64_t ff_workspace_bytes(uint64_t max_pixels, int32_t max_cameras, int32_t max_frames) {
    const Sizes s = sizes_for(max_pixels, max_cameras, max_frames);
    return s.desc + sizeof(BatchState) + sizeof(FrameState) * (uint64_t)max_frames +
           s.px_tiles * (sizeof(TilePart) + 4) + s.counts * (4 * kCountStripes + 9 + sizeof(CamClass)) +
           s.scan * 8 + 2 * s.keys * 12 +
           s.dhist * 4 + kMaxDigits * 4 + s.sort_tiles * 4 + s.cell * 4 + s.keys * 4 +
           sizeof(CamLite) * (uint64_t)max_cameras + (max_pixels + max_cameras + 64) * 4 +
           (max_pixels + 4) * 4 + (uint64_t)kEmcBlocks * 24 + 4096;
}

void ff_context_destroy(ff_context* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    if (c->have_last) (void)hipEventSynchronize(c->last);
    drop_graphs(c);
    for (auto& e : c->tev) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    (void)probe_collect(c, true);
    for (auto& e : c->probe_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (void* p : c->allocs) (void)hipFree(p);
    for (int i = 0; i < kStageSlots; ++i) {
        if (c->h_stage[i]) (void)hipHostFree(c->h_stage[i]);
        if (c->stage_ev[i]) (void)hipEventDestroy(c->stage_ev[i]);
    }
    if (c->last) (void)hipEventDestroy(c->last);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

ff_status ff_context_create(ff_context** out, int device, uint64_t max_pixels,
                            int32_t max_cameras, int32_t max_frames) {
    if (!out) return FF_ERR_INVALID_ARG;
    *out = nullptr;
    if (max_pixels < 1 || max_pixels >= 0xFFFFFFFFull || max_cameras < 1 ||
        max_cameras > kMaxBatchCams || max_frames < 1 || max_frames > kMaxFrames)
        return FF_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return FF_ERR_INVALID_ARG;
    DeviceGuard g(device);
    ff_context* c = new ff_context();
    c->device = device;
    c->max_pixels = max_pixels;
    c->max_cams = max_cameras;
    c->max_frames = max_frames;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
            c->device_name = prop.name;
            c->n_cu = prop.multiProcessorCount;
            for (char& ch : c->device_name)
                if (ch == '"' || ch == '\\') ch = ' ';
        }
        if (c->device_name.empty()) c->device_name = "unknown";
    }
    const Sizes s = sizes_for(max_pixels, max_cameras, max_frames);
    c->desc_bytes = s.desc;
    ff_status st = FF_OK;
    auto fail = [&](ff_status e) { ff_context_destroy(c); return e; };
    if ((st = dalloc(c, (void**)&c->d_desc, s.desc)) != FF_OK) return fail(st);
    for (int i = 0; i < kStageSlots; ++i) {
        if (hipHostMalloc((void**)&c->h_stage[i], s.desc, hipHostMallocDefault) != hipSuccess)
            return fail(FF_ERR_OOM);
        if (hipEventCreateWithFlags(&c->stage_ev[i], hipEventDisableTiming) != hipSuccess)
            return fail(FF_ERR_HIP);
    }
    if (hipEventCreateWithFlags(&c->last, hipEventDisableTiming) != hipSuccess)
        return fail(FF_ERR_HIP);
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(FF_ERR_HIP);
    if ((st = dalloc(c, (void**)&c->bs, sizeof(BatchState))) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->fs, sizeof(FrameState) * max_frames)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->tiles, sizeof(TilePart) * s.px_tiles)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->tile_off, 4 * s.px_tiles)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->counts, s.counts * 4 * kCountStripes)) != FF_OK)
        return fail(st);
    if ((st = dalloc(c, (void**)&c->fine_base, s.counts * 8)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->level, s.counts)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->cls, s.counts * sizeof(CamClass))) != FF_OK) return fail(st);
    c->counts_cap = s.counts;
    if ((st = dalloc(c, (void**)&c->scan_tile, s.scan * 8)) != FF_OK) return fail(st);
    if ((st = dalloc(c, &c->keysA, s.keys * 8)) != FF_OK) return fail(st);
    if ((st = dalloc(c, &c->keysB, s.keys * 8)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->valsA, s.keys * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->valsB, s.keys * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->digit_hist, s.dhist * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->digit_total, kMaxDigits * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->head_cnt, s.sort_tiles * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->cell_start, s.cell * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->conf_sorted, s.keys * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->camlite, sizeof(CamLite) * (size_t)max_cameras)) != FF_OK)
        return fail(st);
    c->raytab_cap = max_pixels + (uint64_t)max_cameras + 64;   // sum of W + H <= P + cameras
    if ((st = dalloc(c, (void**)&c->raytab, c->raytab_cap * 4)) != FF_OK) return fail(st);
    c->sort_tiles_cap = s.sort_tiles;
    if ((st = dalloc(c, (void**)&c->conf_ws, (max_pixels + 4) * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->emc_part, (size_t)kEmcBlocks * 3 * 8)) != FF_OK) return fail(st);
    if (set_smem_limits() != FF_OK) return fail(FF_ERR_HIP);
    *out = c;
    return FF_OK;
}

ff_status ff_get_tuning(const ff_context* c, ff_tuning* t) {
    if (!c || !t) return FF_ERR_INVALID_ARG;
    *t = c->tune;
    return FF_OK;
}

ff_status ff_set_tuning(ff_context* c, const ff_tuning* t) {
    if (!c || !t || !tuning_ok(*t)) return FF_ERR_INVALID_ARG;
    c->tune = *t;              // cached graphs are keyed by their tuning: none goes stale
    return FF_OK;
}

static ff_status fuse_impl(ff_context* c, int32_t n_frames, const ff_frame* frames,
                           const ff_params* params, const ff_output* outs, void* stream,
                           bool batched) {
    if (!c) return FF_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (params && params->coarse_res >= 1 && params->coarse_res <= 128) {
        const uint64_t G = (uint64_t)params->coarse_res;
        ff_status st = grow_counts(c, (uint64_t)std::max(1, n_frames) * G * G * G, s);
        if (st != FF_OK) return st;
    }
    // stage the descriptor in a pinned slot that no queued copy still reads
    const int slot = c->stage;
    c->stage = (c->stage + 1) % kStageSlots;
    FF_HIP(hipEventSynchronize(c->stage_ev[slot]));
    Plan plan;
    std::string shape;
    const ff_tuning T = tuning_for(c, shape_key(n_frames, frames, params));
    ff_status st = build_desc(c, n_frames, frames, params, outs, T, c->h_stage[slot], plan, shape);
    if (st != FF_OK) return st;
    if (c->trace && (st = trace_collect(c)) != FF_OK) return st;
    if (!c->probe_pending.empty() &&
        (st = probe_collect(c, c->probe_pending.size() >= 256)) != FF_OK)
        return st;
    const Ctx C = make_ctx(c);
    // calls on one context share its workspace: order this one after the previous one
    if (c->have_last) FF_HIP(hipStreamWaitEvent(s, c->last, 0));
    FF_HIP(hipMemcpyAsync(c->d_desc, c->h_stage[slot], plan.desc_used, hipMemcpyHostToDevice, s));
    FF_HIP(hipEventRecord(c->stage_ev[slot], s));
    const bool graph = batched && T.use_graph && !c->trace;
    if (c->probe_slot >= 0 && !c->trace) {
        uint64_t px = 0;
        for (int32_t f = 0; f < n_frames; ++f)
            for (int32_t k = 0; k < frames[f].n_cams; ++k)
                px += (uint64_t)frames[f].cams[k].width * (uint64_t)frames[f].cams[k].height;
        st = run_probed(c, C, plan, shape, s, graph, (uint32_t)n_frames, px);
    } else if (graph) {
        st = run_graph(c, C, plan, shape, s);
    } else {
        st = dispatch_plain(c, C, plan, s);
    }
    if (st != FF_OK) return st;
    FF_HIP(hipGetLastError());
    FF_HIP(hipEventRecord(c->last, s));
    c->have_last = true;
    return FF_OK;
}

ff_status ff_fuse(ff_context* c, int32_t n_cams, const ff_camera* cams, const ff_view* views,
                  const ff_params* params, const ff_output* out, void* stream) {
    ff_frame fr{n_cams, cams, views};
    return fuse_impl(c, 1, &fr, params, out, stream, false);
}

ff_status ff_fuse_batch(ff_context* c, int32_t n_frames, const ff_frame* frames,
                        const ff_params* params, const ff_output* outs, void* stream) {
    return fuse_impl(c, n_frames, frames, params, outs, stream, true);
}

void ff_conf_params_default(ff_conf_params* p) {
    if (!p) return;
    p->alpha = 0.5f;
    p->beta = 0.5f;
    p->gamma = 1.0f;
    p->delta = 1.0f;
}

ff_status ff_confidence(int32_t n_cams, const ff_camera* cams, const ff_view* views,
                        float* const* conf_out, const ff_conf_params* prm, void* stream) {
    if (n_cams < 1 || !cams || !views || !conf_out || !prm) return FF_ERR_INVALID_ARG;
    if (!std::isfinite(prm->alpha) || !std::isfinite(prm->beta) || !std::isfinite(prm->gamma) ||
        !std::isfinite(prm->delta) || !(prm->alpha + prm->gamma > 0.0f))
        return FF_ERR_INVALID_ARG;
    for (int32_t k = 0; k < n_cams; ++k) {
        const uint64_t npx = (uint64_t)cams[k].width * (uint64_t)cams[k].height;
        if (cams[k].width < 1 || cams[k].height < 1 || npx >= 0xFFFFFFFFull || !views[k].depth ||
            !conf_out[k])
            return FF_ERR_INVALID_ARG;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const ConfWeights w{prm->alpha, prm->beta, prm->gamma, prm->delta};
    for (int32_t k = 0; k < n_cams; ++k) {
        const uint64_t npx = (uint64_t)cams[k].width * (uint64_t)cams[k].height;
        const dim3 grid((uint32_t)((npx + kBlock - 1) / kBlock)), block(kBlock);
        hipLaunchKernelGGL(k_conf_map, grid, block, 0, s, views[k].depth, conf_out[k],
                           cams[k].width, cams[k].height, w);
    }
    FF_HIP(hipGetLastError());
    return FF_OK;
}

void ff_emc_params_default(ff_emc_params* p) {
    if (!p) return;
    p->c_occ = 0.003f;
    p->stride = 1;
}

ff_status ff_emc(ff_context* c, int32_t n_cams, const ff_camera* cams, const ff_view* views,
                 const float* xyz, const uint32_t* count, uint32_t capacity,
                 const ff_emc_params* prm, double* out, void* stream) {
    if (!c || n_cams < 1 || n_cams > c->max_cams || !cams || !views || !xyz || !count || !prm ||
        !out || prm->stride < 1 || !std::isfinite(prm->c_occ) || prm->c_occ < 0.0f)
        return FF_ERR_INVALID_ARG;
    for (int32_t k = 0; k < n_cams; ++k)
        if (cams[k].width < 1 || cams[k].height < 1 || !views[k].depth) return FF_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // camera records in a pinned staging slot that no queued copy still reads
    const int slot = c->stage;
    c->stage = (c->stage + 1) % kStageSlots;
    FF_HIP(hipEventSynchronize(c->stage_ev[slot]));
    const size_t cam_off = sizeof(CallHdr) + sizeof(DevFrame) * (size_t)c->max_frames;
    DevCam* K = reinterpret_cast<DevCam*>(c->h_stage[slot] + cam_off);
    for (int32_t k = 0; k < n_cams; ++k) {
        DevCam& d = K[k];
        std::memset(&d, 0, sizeof(DevCam));
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) d.R[i * 3 + j] = cams[k].world_to_cam[i * 4 + j];
            d.t[i] = cams[k].world_to_cam[i * 4 + 3];
        }
        d.fx = cams[k].fx; d.fy = cams[k].fy; d.cx = cams[k].cx; d.cy = cams[k].cy;
        d.W = cams[k].width; d.H = cams[k].height;
        d.depth = views[k].depth;
    }
    // calls on one context share its descriptor and workspace: order after the previous one
    if (c->have_last) FF_HIP(hipStreamWaitEvent(s, c->last, 0));
    FF_HIP(hipMemcpyAsync(c->d_desc + cam_off, c->h_stage[slot] + cam_off,
                          sizeof(DevCam) * (size_t)n_cams, hipMemcpyHostToDevice, s));
    FF_HIP(hipEventRecord(c->stage_ev[slot], s));
    const uint64_t m = ((uint64_t)capacity + (uint64_t)prm->stride - 1) / (uint64_t)prm->stride;
    const int nb = (int)std::max<uint64_t>(1, std::min<uint64_t>(kEmcBlocks, (m + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_emc, dim3(nb), dim3(kBlock), 0, s,
                       reinterpret_cast<const DevCam*>(c->d_desc + cam_off), n_cams, xyz, count,
                       capacity, prm->c_occ, (uint32_t)prm->stride, c->emc_part);
    hipLaunchKernelGGL(k_emc_final, dim3(1), dim3(kBlock), 0, s, c->emc_part, nb, out);
    FF_HIP(hipGetLastError());
    FF_HIP(hipEventRecord(c->last, s));
    c->have_last = true;
    return FF_OK;
}

}  // extern "C"

namespace {

// Device address of `scratch` on each device, taken once per device with that device
// current (in host code the array's name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

ff_status scratch_on_current_device(char** out) {
    int dev = -1;
    FF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return FF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        FF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return FF_ERR_HIP;
        g_scratch[dev] = static_cast<char*>(p);
    }
    *out = g_scratch[dev];
    return FF_OK;
}

}  // namespace

extern "C" {

ff_status ff_emc_noalloc(int32_t n_cams, const ff_camera* cams, const ff_view* views,
                         const float* xyz, const uint32_t* count, uint32_t capacity,
                         const ff_emc_params* prm, double* out, void* stream) {
    if (n_cams < 1 || !cams || !views || !xyz || !count || !prm || !out || prm->stride < 1 ||
        !std::isfinite(prm->c_occ) || prm->c_occ < 0.0f)
        return FF_ERR_INVALID_ARG;
    if (n_cams > kNoAllocMaxCams) return FF_ERR_INVALID_ARG;     // beyond the scratch table
    for (int32_t k = 0; k < n_cams; ++k)
        if (cams[k].width < 1 || cams[k].height < 1 || !views[k].depth) return FF_ERR_INVALID_ARG;
    char* base = nullptr;
    ff_status st = scratch_on_current_device(&base);
    if (st != FF_OK) return st;
    DevCam* dcams = reinterpret_cast<DevCam*>(base);
    double* part = reinterpret_cast<double*>(base + kNoAllocCamBytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (int32_t b = 0; b < n_cams; b += kNoAllocCamsPerLaunch) {
        EmcCamChunk chunk{};
        const int n = std::min<int32_t>(kNoAllocCamsPerLaunch, n_cams - b);
        for (int k = 0; k < n; ++k) {
            const ff_camera& c = cams[b + k];
            EmcCamArgs& a = chunk.cam[k];
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) a.R[i * 3 + j] = c.world_to_cam[i * 4 + j];
                a.t[i] = c.world_to_cam[i * 4 + 3];
            }
            a.fx = c.fx; a.fy = c.fy; a.cx = c.cx; a.cy = c.cy;
            a.W = c.width; a.H = c.height;
            a.depth = views[b + k].depth;
        }
        hipLaunchKernelGGL(k_emc_cams, dim3(1), dim3(64), 0, s, chunk, dcams, (int)b, n);
    }
    const uint64_t m = ((uint64_t)capacity + (uint64_t)prm->stride - 1) / (uint64_t)prm->stride;
    const int nb = (int)std::max<uint64_t>(1, std::min<uint64_t>(kEmcBlocks, (m + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_emc, dim3(nb), dim3(kBlock), 0, s, dcams, n_cams, xyz, count, capacity,
                       prm->c_occ, (uint32_t)prm->stride, part);
    hipLaunchKernelGGL(k_emc_final, dim3(1), dim3(kBlock), 0, s, part, nb, out);
    FF_HIP(hipGetLastError());
    return FF_OK;
}

ff_status ff_trace_enable(ff_context* c, int32_t on) {
    if (!c) return FF_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    if (c->trace) {
        ff_status st = trace_collect(c);
        if (st != FF_OK) return st;
    }
    c->trace = on != 0;
    c->tacc = ff_trace{};
    return FF_OK;
}

ff_status ff_trace_read(ff_context* c, ff_trace* out) {
    if (!c || !out) return FF_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    ff_status st = trace_collect(c);
    *out = c->tacc;
    return st;
}

ff_status ff_probe_enable(ff_context* c, int32_t slot) {
    if (!c || slot < -1 || slot >= FF_TRACE_SLOTS) return FF_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    ff_status st = probe_collect(c, true);
    c->probe_slot = slot;
    c->pacc = ff_probe{};
    c->pacc.slot = slot;
    return st;
}

ff_status ff_probe_read(ff_context* c, ff_probe* out) {
    if (!c || !out) return FF_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    ff_status st = probe_collect(c, true);
    *out = c->pacc;
    return st;
}

const char* ff_trace_slot_name(int32_t slot) {
    static const char* names[] = {"backproject_aabb", "tile_reduce", "coarse_hist",
                                  "coarse_scan_a", "coarse_scan_m", "coarse_scan_b", "keys",
                                  "camera_classes", "radix_scan", "radix_down", "head_count",
                                  "head_scan", "head_write", "cells_top3_consistency_fuse",
                                  "final", "cam_prep"};
    if (slot >= 0 && slot < 16) return names[slot];
    static const char* radix[] = {"radix_up_p0", "radix_scan_p0", "radix_down_p0",
                                  "radix_up_p1", "radix_scan_p1", "radix_down_p1",
                                  "radix_up_p2", "radix_scan_p2", "radix_down_p2",
                                  "radix_up_p3", "radix_scan_p3", "radix_down_p3",
                                  "radix_up_p4", "radix_scan_p4", "radix_down_p4+",
                                  "confidence_eq3"};
    if (slot >= 16 && slot < 32) return radix[slot - 16];
    return "unused";
}

ff_status ff_autotune(ff_context* c, int32_t n_frames, const ff_frame* frames,
                      const ff_params* params, const ff_output* outs, void* stream,
                      ff_tuning* chosen) {
    if (!c) return FF_ERR_INVALID_ARG;
    const std::string key = shape_key(n_frames, frames, params);
    if (key.empty()) return FF_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool had = c->tuned.count(key) != 0;
    const ff_tuning keep = tuning_for(c, key);
    hipEvent_t e0, e1;
    FF_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FF_ERR_HIP;
    }
    ff_status st = FF_OK;
    // one untimed and three timed calls of the batch with candidate t cached for its shape
    auto time_of = [&](const ff_tuning& t, float& ms) -> ff_status {
        c->tuned[key] = t;
        ff_status r = ff_fuse_batch(c, n_frames, frames, params, outs, stream);
        if (r != FF_OK) return r;
        FF_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < 3 && r == FF_OK; ++i)
            r = ff_fuse_batch(c, n_frames, frames, params, outs, stream);
        if (r != FF_OK) return r;
        FF_HIP(hipEventRecord(e1, s));
        FF_HIP(hipEventSynchronize(e1));
        FF_HIP(hipEventElapsedTime(&ms, e0, e1));
        return FF_OK;
    };
    ff_tuning best = keep;
    float best_ms = 1e30f;
    // one knob at a time: digit width x keys per thread, then histogram tiles per
    // workgroup, then per-cell workgroups
    for (int b : {6, 7, 8, 9, 10}) {
        for (int it : {8, 16}) {
            ff_tuning t = best;
            t.radix_bits = b;
            t.sort_items = it;
            float ms = 0.0f;
            if ((st = time_of(t, ms)) != FF_OK) break;
            if (ms < best_ms) { best_ms = ms; best = t; }
        }
        if (st != FF_OK) break;
    }
    const ff_tuning after_sort = best;
    for (int h : {0, 1, 2, 4, 8}) {
        if (st != FF_OK) break;
        ff_tuning t = after_sort;
        t.hist_tiles = h;
        float ms = 0.0f;
        if ((st = time_of(t, ms)) != FF_OK) break;
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    const ff_tuning after_hist = best;
    for (int cg : {0, 768, 1024, 1280, 2048, 2560, 3840}) {
        if (st != FF_OK) break;
        ff_tuning t = after_hist;
        t.cell_groups = cg;
        float ms = 0.0f;
        if ((st = time_of(t, ms)) != FF_OK) break;
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == FF_OK) {
        c->tuned[key] = best;
    } else if (had) {
        c->tuned[key] = keep;
    } else {
        c->tuned.erase(key);
    }
    if (chosen) *chosen = st == FF_OK ? best : keep;
    return st;
}

}  // extern "C"

void ff::share_tuning(const ff_context* src, ff_context* dst) {
    if (!src || !dst || src == dst) return;
    for (const auto& kv : src->tuned) dst->tuned[kv.first] = kv.second;
}

extern "C" {

ff_status ff_tuning_lookup(const ff_context* c, int32_t n_frames, const ff_frame* frames,
                           const ff_params* params, ff_tuning* t, int32_t* found) {
    if (!c || !t || !found) return FF_ERR_INVALID_ARG;
    const std::string key = shape_key(n_frames, frames, params);
    if (key.empty()) return FF_ERR_INVALID_ARG;
    auto it = c->tuned.find(key);
    *found = it != c->tuned.end() ? 1 : 0;
    if (*found) *t = it->second;
    return FF_OK;
}

ff_status ff_tuning_export(const ff_context* c, char* buf, uint64_t cap, uint64_t* needed) {
    if (!c || !needed || (cap > 0 && !buf)) return FF_ERR_INVALID_ARG;
    std::string j = "{\"device\": \"" + c->device_name + "\", \"entries\": [";
    char tmp[160];
    bool first = true;
    for (const auto& kv : c->tuned) {
        const ff_tuning& t = kv.second;
        std::snprintf(tmp, sizeof(tmp),
                      "\", \"radix_bits\": %d, \"sort_items\": %d, \"hist_tiles\": %d, "
                      "\"cell_groups\": %d, \"use_graph\": %d}",
                      t.radix_bits, t.sort_items, t.hist_tiles, t.cell_groups, t.use_graph);
        j += std::string(first ? "" : ", ") + "{\"shape\": \"" + kv.first + tmp;
        first = false;
    }
    j += "]}";
    *needed = j.size() + 1;
    if (cap < j.size() + 1) return FF_ERR_INVALID_ARG;
    std::memcpy(buf, j.c_str(), j.size() + 1);
    return FF_OK;
}

namespace {

// the string value following "name": in text at or after pos (no escapes: device names
// and shape keys contain none); npos when absent
size_t json_string(const std::string& text, const char* name, size_t pos, std::string& out) {
    const std::string pat = std::string("\"") + name + "\"";
    size_t k = text.find(pat, pos);
    if (k == std::string::npos) return k;
    k = text.find(':', k + pat.size());
    if (k == std::string::npos) return k;
    k = text.find('"', k);
    if (k == std::string::npos) return k;
    const size_t e = text.find('"', k + 1);
    if (e == std::string::npos) return e;
    out = text.substr(k + 1, e - k - 1);
    return e + 1;
}

bool json_int(const std::string& obj, const char* name, int32_t& out) {
    const std::string pat = std::string("\"") + name + "\"";
    size_t k = obj.find(pat);
    if (k == std::string::npos) return false;
    k = obj.find(':', k + pat.size());
    if (k == std::string::npos) return false;
    char* end = nullptr;
    const long v = std::strtol(obj.c_str() + k + 1, &end, 10);
    if (end == obj.c_str() + k + 1 || v < -1000000 || v > 1000000) return false;
    out = (int32_t)v;
    return true;
}

}  // namespace

ff_status ff_tuning_import(ff_context* c, const char* json, int32_t* imported) {
    if (!c || !json) return FF_ERR_INVALID_ARG;
    const std::string text(json);
    std::string dev;
    if (json_string(text, "device", 0, dev) == std::string::npos) return FF_ERR_INVALID_ARG;
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos) return FF_ERR_INVALID_ARG;
    std::vector<std::pair<std::string, ff_tuning>> got;
    while (true) {
        const size_t ob = text.find('{', pos);
        if (ob == std::string::npos) break;
        const size_t cb = text.find('}', ob);
        if (cb == std::string::npos) return FF_ERR_INVALID_ARG;
        const std::string obj = text.substr(ob, cb - ob + 1);
        std::string shape;
        ff_tuning t{};
        if (json_string(obj, "shape", 0, shape) == std::string::npos ||
            !json_int(obj, "radix_bits", t.radix_bits) || !json_int(obj, "sort_items", t.sort_items) ||
            !json_int(obj, "hist_tiles", t.hist_tiles) ||
            !json_int(obj, "cell_groups", t.cell_groups) || !json_int(obj, "use_graph", t.use_graph) ||
            !tuning_ok(t) || shape.empty())
            return FF_ERR_INVALID_ARG;
        got.emplace_back(shape, t);
        pos = cb + 1;
    }
    int32_t n = 0;
    if (dev == c->device_name) {
        for (const auto& e : got) c->tuned[e.first] = e.second;
        n = (int32_t)got.size();
    }
    if (imported) *imported = n;
    return FF_OK;
}

}  // extern "C"
