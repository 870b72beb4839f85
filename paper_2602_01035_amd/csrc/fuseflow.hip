// Host library and kernels of the fusion path (C ABI in include/fuseflow.h).
//
// Launch structure: a prep kernel clears the per-call state, then one kernel per phase of
// phases.hpp runs over every frame of the call (workgroups claim work items with a ticket
// counter, so items start in increasing order).  ff_fuse enqueues the kernels directly;
// ff_fuse_batch replays them from a HIP graph cached per batch shape.
//
// A single persistent launch running all phases (k_persistent, FF_EXPERIMENTAL_PERSISTENT)
// is kept out of the build: it did not finish on the device and its cause is not known.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fuseflow.h"
#include "common.hpp"
#include "phases.hpp"

using namespace ff;

// ============================================================================ kernels

// Clears the per-call state, bumps the look-back epoch and derives each camera's centre
// c = -R^T t (canonical order) and its rank under (centre x, y, z, index) in its frame.
__global__ __launch_bounds__(kBlock) void k_prep(Ctx C, uint32_t n_counts, int bump_epoch) {
    const CallHdr& H = *C.hdr;
    const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
    for (uint32_t i = gtid; i < n_counts; i += gridDim.x * kBlock) C.counts[i] = 0;
    if (blockIdx.x != 0) return;
    BatchState* bs = C.bs;
    uint32_t* words = reinterpret_cast<uint32_t*>(bs);
    for (uint32_t i = threadIdx.x; i < sizeof(BatchState) / 4; i += kBlock) words[i] = 0;
    for (uint32_t f = threadIdx.x; f < H.n_frames; f += kBlock) {
        FrameState& st = C.fs[f];
        for (int a = 0; a < 3; ++a) { st.bmin_o[a] = 0xFFFFFFFFu; st.bmax_o[a] = 0u; }
        st.M = st.S = st.R = 0;
        st.fine_begin = 0;
    }
    for (uint32_t i = threadIdx.x; i < H.n_cams; i += kBlock) {
        DevCam& cm = C.cams[i];
        for (int a = 0; a < 3; ++a)
            cm.c[a] = -((cm.R[0 * 3 + a] * cm.t[0] + cm.R[1 * 3 + a] * cm.t[1]) +
                        cm.R[2 * 3 + a] * cm.t[2]);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < H.n_cams; i += kBlock) {
        DevCam& cm = C.cams[i];
        const DevFrame& fr = C.frames[cm.frame];
        uint32_t rk = 0;
        for (uint32_t j = fr.cam_begin; j < fr.cam_begin + fr.n_cams; ++j) {
            const DevCam& o = C.cams[j];
            bool before;
            if (o.c[0] != cm.c[0]) before = o.c[0] < cm.c[0];
            else if (o.c[1] != cm.c[1]) before = o.c[1] < cm.c[1];
            else if (o.c[2] != cm.c[2]) before = o.c[2] < cm.c[2];
            else before = j < i;
            rk += before ? 1u : 0u;
        }
        cm.rank = rk;
    }
    if (threadIdx.x == 0 && bump_epoch) *const_cast<uint32_t*>(C.epoch) += 1u;
}

template <int ITEMS>
__device__ __forceinline__ void run_phase(const Ctx& C, uint32_t kind, uint32_t item,
                                          char* smem) {
    switch (kind) {
        case PH_BACKPROJECT: ph_backproject(C, item, smem); break;
        case PH_HIST: ph_hist(C, item, smem); break;
        case PH_SCAN_A: ph_scan_a(C, item, smem); break;
        case PH_SCAN_M: ph_scan_m(C, item, smem); break;
        case PH_SCAN_B: ph_scan_b(C, item, smem); break;
        case PH_KEYS: ph_keys(C, item, smem); break;
        case PH_HEADS: ph_heads<ITEMS>(C, item, smem); break;
        case PH_CELLS: ph_cells(C, item, smem); break;
        case PH_FINAL: ph_final(C, item, smem); break;
        default: ph_radix<ITEMS>(C, kind - PH_RADIX, item, smem); break;
    }
}

// One phase per launch: workgroups claim items with the phase's ticket counter, so items
// are started in increasing order (the look-back of an item only waits on started items).
template <int KIND, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_phase(Ctx C, uint32_t slot, uint32_t n_items,
                                                  uint32_t pass) {
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t s_t;
    while (true) {
        if (threadIdx.x == 0) s_t = atomicAdd(&C.bs->tickets[slot], 1u);
        __syncthreads();
        const uint32_t t = s_t;
        __syncthreads();
        if (t >= n_items) break;
        if (KIND == PH_RADIX) ph_radix<ITEMS>(C, pass, t, smem);
        else run_phase<ITEMS>(C, KIND, t, smem);
        __syncthreads();
    }
}

#ifdef FF_EXPERIMENTAL_PERSISTENT
// All phases in one launch.  Tickets are global and phase-ordered; before an item runs,
// its workgroup waits until every item of the previous phase has completed.  A waiting
// workgroup only ever waits on items claimed before its own, which are held by running
// workgroups, so the launch needs no co-residency guarantee.
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_persistent(Ctx C) {
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t s_t;
    const CallHdr& H = *C.hdr;
    const uint32_t n_phases = H.n_phases;
    const uint32_t total = H.phase_begin[n_phases];
    BatchState* bs = C.bs;
    while (true) {
        if (threadIdx.x == 0) s_t = atomicAdd(&bs->tickets[0], 1u);
        __syncthreads();
        const uint32_t t = s_t;
        __syncthreads();
        if (t >= total) break;
        uint32_t p = 0;
        while (p + 1 < n_phases && H.phase_begin[p + 1] <= t) ++p;
        if (p > 0 && threadIdx.x == 0) {
            // poll with relaxed loads (an acquire per poll would invalidate the L2 each
            // time and starve the workgroups doing the work), then acquire once
            const uint32_t need = H.phase_begin[p] - H.phase_begin[p - 1];
            Waiter wt(H.wait_ticks);
            while (ld_relaxed(&bs->done[p - 1]) < need) {
                if (wt.expired(bs)) {
                    raise_error(bs, kErrSpin);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        run_phase<ITEMS>(C, H.phase_kind[p], t - H.phase_begin[p], smem);
        // each wave makes its own stores visible device-wide before the item is counted
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&bs->done[p], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}
#endif  // FF_EXPERIMENTAL_PERSISTENT

__global__ void k_fill_u64(uint64_t* p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ============================================================================ host side

namespace {

constexpr int kStageSlots = 4;

size_t radix_smem(int items) {
    const size_t kt = (size_t)kBlock * items;
    return kt * 8 + kt * 4 + (4 + 2) * kMaxDigits * 4 + 64;
}
size_t keys_smem() { return (8 + kMaxPass * kMaxDigits + 8) * 4; }
size_t cells_smem() { return sizeof(CellsShared); }
size_t phase_smem(int items) {
    return std::max({radix_smem(items), keys_smem(), cells_smem(), (size_t)4096});
}

struct Buf {
    void* p = nullptr;
    size_t n = 0;
};

int ilog2(uint32_t v) {
    int r = 0;
    while ((1u << r) < v) ++r;
    return r;
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
    uint32_t* counts = nullptr;
    uint64_t* fine_base = nullptr;
    uint64_t counts_cap = 0;
    uint64_t* scan_tile = nullptr;
    uint64_t scan_cap = 0;
    void* keysA = nullptr;
    void* keysB = nullptr;
    uint32_t* valsA = nullptr;
    uint32_t* valsB = nullptr;
    uint32_t* cell_start = nullptr;
    uint64_t* lb_tile = nullptr;
    uint64_t* lb_digit = nullptr;
    uint64_t lb_tile_cap = 0, lb_digit_cap = 0;
    uint32_t* epoch = nullptr;
    uint64_t calls = 0;
    hipEvent_t last = nullptr;
    bool have_last = false;
    std::vector<void*> allocs;
    ff_tuning tune{8, 8, 256, 1};
    hipStream_t cap_stream = nullptr;
    uint64_t wait_ticks = 200000000ull;   // 2 s at the 100 MHz wall clock
    std::map<std::string, hipGraphExec_t> graphs;
    // kernel tracing (events on the call's stream)
    bool trace = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;   // per launch of the pending call
    std::vector<int> tslot;
    size_t tused = 0;
    ff_trace tacc{};
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
            last_hip_error() = e_;                      \
            return FF_ERR_HIP;                          \
        }                                               \
    } while (0)

hipError_t& last_hip_error() {
    static thread_local hipError_t e = hipSuccess;
    return e;
}

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

uint64_t n_lb_digit(uint64_t P, int items) {
    const uint64_t kt = (uint64_t)kBlock * items;
    return ((P + kt - 1) / kt + 1) * kMaxDigits;
}

// All sizes that depend only on the context limits.
struct Sizes {
    uint64_t desc, counts, scan, keys, vals, cell, lbt, lbd;
};
Sizes sizes_for(uint64_t P, int32_t C, int32_t F) {
    Sizes s;
    s.desc = sizeof(CallHdr) + sizeof(DevFrame) * (uint64_t)F + sizeof(DevCam) * (uint64_t)C;
    s.counts = (uint64_t)F * 64 * 64 * 64;           // grows on demand for coarse_res > 64
    s.scan = (s.counts + kScanTile - 1) / kScanTile + 1;
    s.keys = P + 1;
    s.vals = P + 1;
    s.cell = P + 2;
    s.lbt = (P + 1023) / 1024 + 64;
    s.lbd = n_lb_digit(P, 4);
    return s;
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
    if (p->flags & ~7u) return FF_ERR_INVALID_ARG;
    return FF_OK;
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
    drop(c->scan_tile);
    c->counts = nullptr; c->fine_base = nullptr; c->scan_tile = nullptr;
    ff_status st;
    if ((st = dalloc(c, (void**)&c->counts, need * 4)) != FF_OK) return st;
    if ((st = dalloc(c, (void**)&c->fine_base, need * 8)) != FF_OK) return st;
    c->scan_cap = (need + kScanTile - 1) / kScanTile + 1;
    if ((st = dalloc(c, (void**)&c->scan_tile, c->scan_cap * 8)) != FF_OK) return st;
    c->counts_cap = need;
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);   // captured old pointers
    c->graphs.clear();
    return FF_OK;
}

Ctx make_ctx(ff_context* c) {
    Ctx C;
    C.hdr = reinterpret_cast<const CallHdr*>(c->d_desc);
    C.frames = reinterpret_cast<const DevFrame*>(c->d_desc + sizeof(CallHdr));
    C.cams = reinterpret_cast<DevCam*>(c->d_desc + sizeof(CallHdr) +
                                       sizeof(DevFrame) * (size_t)c->max_frames);
    C.bs = c->bs;
    C.fs = c->fs;
    C.counts = c->counts;
    C.fine_base = c->fine_base;
    C.scan_tile = c->scan_tile;
    C.keysA = c->keysA;
    C.keysB = c->keysB;
    C.valsA = c->valsA;
    C.valsB = c->valsB;
    C.cell_start = c->cell_start;
    C.lb_tile = c->lb_tile;
    C.lb_digit = c->lb_digit;
    C.epoch = c->epoch;
    C.P_cap = (uint32_t)std::min<uint64_t>(c->max_pixels, 0xFFFFFFFEull);
    C.lb_tile_cap = (uint32_t)c->lb_tile_cap;
    C.lb_digit_cap = (uint32_t)std::min<uint64_t>(c->lb_digit_cap, 0xFFFFFFFFull);
    return C;
}

struct Plan {
    std::vector<std::pair<uint32_t, uint32_t>> phases;   // (kind, n_items)
    uint32_t n_counts = 0;
};

// Validate one batch and fill the host staging descriptor.  Returns the launch plan.
ff_status build_desc(ff_context* c, int32_t n_frames, const ff_frame* frames,
                     const ff_params* prm, const ff_output* outs, char* stage, Plan& plan,
                     std::string& shape) {
    if (n_frames < 1 || n_frames > c->max_frames || !frames || !outs) return FF_ERR_INVALID_ARG;
    ff_status st = validate_params(prm);
    if (st != FF_OK) return st;
    CallHdr* H = reinterpret_cast<CallHdr*>(stage);
    DevFrame* F = reinterpret_cast<DevFrame*>(stage + sizeof(CallHdr));
    DevCam* K = reinterpret_cast<DevCam*>(stage + sizeof(CallHdr) +
                                          sizeof(DevFrame) * (size_t)c->max_frames);
    std::memset(H, 0, sizeof(CallHdr));
    uint64_t P = 0;
    uint32_t ncam = 0, ntile = 0;
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
            if (cm.width < 1 || cm.height < 1 || !v.depth || !v.conf) return FF_ERR_INVALID_ARG;
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
            d.vec_ok = ((uintptr_t)v.depth % 16 == 0 && (uintptr_t)v.conf % 16 == 0) ? 1u : 0u;
            d.depth = v.depth;
            d.conf = v.conf;
            d.rgb = v.rgb;
            all_rgb = all_rgb && v.rgb;
            ntile += (uint32_t)((npx + kPxTile - 1) / kPxTile);
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
    H->wait_ticks = c->wait_ticks;
    H->n_frames = (uint32_t)n_frames;
    H->n_cams = ncam;
    H->n_px_tiles = ntile;
    H->P_tot = (uint32_t)P;
    const uint64_t ncounts = (uint64_t)n_frames * G3;
    H->n_scan_tiles = (uint32_t)((ncounts + kScanTile - 1) / kScanTile);
    const uint32_t KT = (uint32_t)(kBlock * c->tune.sort_items);
    H->n_sort_tiles = (uint32_t)((P + KT - 1) / KT);
    H->n_cell_items = (uint32_t)std::min<uint64_t>(4096, std::max<uint64_t>(1, (P + 2047) / 2048));
    H->radix_bits = (uint32_t)c->tune.radix_bits;
    // widest possible dense key: frames x coarse cells x 8^Lmax
    const uint32_t bits_max = (uint32_t)(ilog2((uint32_t)n_frames) + 3 * H->prm.log2G +
                                         3 * prm->max_level);
    H->npass_max = (bits_max + H->radix_bits - 1) / H->radix_bits;
    if (H->npass_max > (uint32_t)kMaxPass) return FF_ERR_INVALID_ARG;
    const bool no_sa = prm->flags & FF_NO_SA;
    plan.phases.clear();
    plan.phases.push_back({PH_BACKPROJECT, ntile});
    if (!no_sa) {
        plan.phases.push_back({PH_HIST, ntile});
        plan.phases.push_back({PH_SCAN_A, H->n_scan_tiles});
        plan.phases.push_back({PH_SCAN_M, 1});
        plan.phases.push_back({PH_SCAN_B, H->n_scan_tiles});
    }
    plan.phases.push_back({PH_KEYS, ntile});
    if (!no_sa) {
        for (uint32_t k = 0; k < H->npass_max; ++k)
            plan.phases.push_back({PH_RADIX + k, H->n_sort_tiles});
        plan.phases.push_back({PH_HEADS, H->n_sort_tiles});
    }
    plan.phases.push_back({PH_CELLS, H->n_cell_items});
    plan.phases.push_back({PH_FINAL, 1});
    H->n_phases = (uint32_t)plan.phases.size();
    uint32_t acc = 0;
    for (size_t i = 0; i < plan.phases.size(); ++i) {
        H->phase_begin[i] = acc;
        H->phase_kind[i] = plan.phases[i].first;
        acc += plan.phases[i].second;
    }
    H->phase_begin[plan.phases.size()] = acc;
    plan.n_counts = no_sa ? 0u : (uint32_t)ncounts;
    char tail[96];
    std::snprintf(tail, sizeof(tail), "|G%d|L%d|f%u|t%d,%d", G, prm->max_level, prm->flags,
                  c->tune.radix_bits, c->tune.sort_items);
    shape += tail;
    return FF_OK;
}

template <int ITEMS>
void launch_phase(const Ctx& C, uint32_t kind, uint32_t slot, uint32_t n, size_t smem,
                  hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(n, 2048));
#define FF_L(K) hipLaunchKernelGGL((k_phase<K, ITEMS>), dim3(grid), dim3(kBlock), smem, s, C, slot, n, 0u)
    switch (kind) {
        case PH_BACKPROJECT: FF_L(PH_BACKPROJECT); break;
        case PH_HIST: FF_L(PH_HIST); break;
        case PH_SCAN_A: FF_L(PH_SCAN_A); break;
        case PH_SCAN_M: FF_L(PH_SCAN_M); break;
        case PH_SCAN_B: FF_L(PH_SCAN_B); break;
        case PH_KEYS: FF_L(PH_KEYS); break;
        case PH_HEADS: FF_L(PH_HEADS); break;
        case PH_CELLS: FF_L(PH_CELLS); break;
        case PH_FINAL: FF_L(PH_FINAL); break;
        default:
            hipLaunchKernelGGL((k_phase<PH_RADIX, ITEMS>), dim3(grid), dim3(kBlock), smem, s, C,
                               slot, n, kind - PH_RADIX);
    }
#undef FF_L
}

size_t smem_for(uint32_t kind, int items) {
    switch (kind) {
        case PH_KEYS: return keys_smem();
        case PH_CELLS: return cells_smem();
        case PH_HEADS: return 4096;
        case PH_BACKPROJECT: case PH_HIST: case PH_FINAL: return 64;
        case PH_SCAN_A: case PH_SCAN_M: case PH_SCAN_B: return 256;
        default: return radix_smem(items);
    }
}

// Stage the descriptor and order this call after the previous one on the workspace.
ff_status begin_call(ff_context* c, hipStream_t s, char** stage) {
    const int slot = c->stage;
    c->stage = (c->stage + 1) % kStageSlots;
    FF_HIP(hipEventSynchronize(c->stage_ev[slot]));
    *stage = c->h_stage[slot];
    return FF_OK;
}

ff_status submit_desc(ff_context* c, hipStream_t s, const Ctx& C, const Plan& plan,
                      bool use_graph_kernels) {
    const int slot = (c->stage + kStageSlots - 1) % kStageSlots;
    if (c->have_last) FF_HIP(hipStreamWaitEvent(s, c->last, 0));
    FF_HIP(hipMemcpyAsync(c->d_desc, c->h_stage[slot], c->desc_bytes, hipMemcpyHostToDevice, s));
    FF_HIP(hipEventRecord(c->stage_ev[slot], s));
    // look-back words carry a 30-bit tag built from the epoch; clear them before it wraps
    if ((++c->calls & ((1ull << 24) - 1)) == 0) {
        hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, c->lb_tile, c->lb_tile_cap);
        hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, c->lb_digit, c->lb_digit_cap);
    }
    (void)C; (void)plan; (void)use_graph_kernels;
    return FF_OK;
}

ff_status end_call(ff_context* c, hipStream_t s) {
    FF_HIP(hipGetLastError());
    FF_HIP(hipEventRecord(c->last, s));
    c->have_last = true;
    return FF_OK;
}

int trace_slot(uint32_t kind) {
    switch (kind) {
        case PH_BACKPROJECT: return 1;
        case PH_HIST: return 2;
        case PH_SCAN_A: return 3;
        case PH_SCAN_M: return 4;
        case PH_SCAN_B: return 5;
        case PH_KEYS: return 6;
        case PH_HEADS: return 7;
        case PH_CELLS: return 8;
        case PH_FINAL: return 9;
        default: return 16 + (int)(kind - PH_RADIX);
    }
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

template <int ITEMS>
ff_status run_plain(ff_context* c, const Ctx& C, const Plan& plan, hipStream_t s) {
    const bool tr = c->trace;
    const uint32_t nc = plan.n_counts;
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(1024, (nc + 4 * kBlock - 1) / (4 * kBlock)));
    if (tr) { ff_status st = trace_mark(c, 0, true, s); if (st != FF_OK) return st; }
    hipLaunchKernelGGL(k_prep, dim3(grid), dim3(kBlock), 0, s, C, nc, 1);
    if (tr) { ff_status st = trace_mark(c, 0, false, s); if (st != FF_OK) return st; }
    for (size_t i = 0; i < plan.phases.size(); ++i) {
        const uint32_t kind = plan.phases[i].first;
        if (tr) { ff_status st = trace_mark(c, trace_slot(kind), true, s); if (st != FF_OK) return st; }
        launch_phase<ITEMS>(C, kind, (uint32_t)i + 1, plan.phases[i].second,
                            smem_for(kind, ITEMS), s);
        if (tr) { ff_status st = trace_mark(c, trace_slot(kind), false, s); if (st != FF_OK) return st; }
    }
    FF_HIP(hipGetLastError());
    return FF_OK;
}

ff_status dispatch_plain(ff_context* c, const Ctx& C, const Plan& plan, hipStream_t s) {
    switch (c->tune.sort_items) {
        case 4: return run_plain<4>(c, C, plan, s);
        case 16: return run_plain<16>(c, C, plan, s);
        default: return run_plain<8>(c, C, plan, s);
    }
}

// Replay the batch's kernels from a graph captured once per shape (resolution mix,
// frame count, grid parameters and tuning): one launch per batch on the stream.
ff_status run_graph(ff_context* c, const Ctx& C, const Plan& plan, const std::string& key,
                    hipStream_t s) {
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        if (c->graphs.size() >= 64) {
            FF_HIP(hipStreamSynchronize(s));
            for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
            c->graphs.clear();
        }
        hipGraph_t g = nullptr;
        FF_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        ff_status st = dispatch_plain(c, C, plan, c->cap_stream);
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (st != FF_OK) { if (g) (void)hipGraphDestroy(g); return st; }
        FF_HIP(e);
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        FF_HIP(e);
        it = c->graphs.emplace(key, ex).first;
    }
    FF_HIP(hipGraphLaunch(it->second, s));
    return FF_OK;
}

ff_status set_smem_limits() {
    static std::once_flag once;
    static ff_status result = FF_OK;
    std::call_once(once, [] {
        auto setk = [](const void* f, size_t b) {
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b) != hipSuccess)
                result = FF_ERR_HIP;
        };
        setk((const void*)k_phase<PH_RADIX, 4>, radix_smem(4));
        setk((const void*)k_phase<PH_RADIX, 8>, radix_smem(8));
        setk((const void*)k_phase<PH_RADIX, 16>, radix_smem(16));
        setk((const void*)k_phase<PH_CELLS, 4>, cells_smem());
        setk((const void*)k_phase<PH_CELLS, 8>, cells_smem());
        setk((const void*)k_phase<PH_CELLS, 16>, cells_smem());
    });
    return result;
}

}  // namespace

// ============================================================================ C ABI

extern "C" {

const char* ff_version(void) { return "fuseflow-mi355x 0.1 (gfx950)"; }

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
           s.counts * 12 + s.scan * 8 + 2 * s.keys * 8 + 2 * s.vals * 4 + s.cell * 4 +
           (s.lbt + s.lbd) * 8 + 256;
}

void ff_context_destroy(ff_context* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    if (c->have_last) (void)hipEventSynchronize(c->last);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& e : c->tev) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
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
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return FF_ERR_INVALID_ARG;
    if (max_pixels < 1 || max_pixels >= 0xFFFFFFFFull || max_cameras < 1 ||
        max_cameras > kMaxBatchCams || max_frames < 1 || max_frames > kMaxFrames)
        return FF_ERR_INVALID_ARG;
    DeviceGuard g(device);
    ff_context* c = new ff_context();
    c->device = device;
    c->max_pixels = max_pixels;
    c->max_cams = max_cameras;
    c->max_frames = max_frames;
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
    if ((st = dalloc(c, (void**)&c->counts, s.counts * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->fine_base, s.counts * 8)) != FF_OK) return fail(st);
    c->counts_cap = s.counts;
    if ((st = dalloc(c, (void**)&c->scan_tile, s.scan * 8)) != FF_OK) return fail(st);
    c->scan_cap = s.scan;
    if ((st = dalloc(c, &c->keysA, s.keys * 8)) != FF_OK) return fail(st);
    if ((st = dalloc(c, &c->keysB, s.keys * 8)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->valsA, s.vals * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->valsB, s.vals * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->cell_start, s.cell * 4)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->lb_tile, s.lbt * 8)) != FF_OK) return fail(st);
    if ((st = dalloc(c, (void**)&c->lb_digit, s.lbd * 8)) != FF_OK) return fail(st);
    c->lb_tile_cap = s.lbt;
    c->lb_digit_cap = s.lbd;
    if ((st = dalloc(c, (void**)&c->epoch, 256)) != FF_OK) return fail(st);
    if (hipMemset(c->lb_tile, 0, s.lbt * 8) != hipSuccess ||
        hipMemset(c->lb_digit, 0, s.lbd * 8) != hipSuccess ||
        hipMemset(c->epoch, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return fail(FF_ERR_HIP);
    if (set_smem_limits() != FF_OK) return fail(FF_ERR_HIP);
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        c->wait_ticks = (uint64_t)khz * 2000ull;   // 2 s
    *out = c;
    return FF_OK;
}

ff_status ff_get_tuning(const ff_context* c, ff_tuning* t) {
    if (!c || !t) return FF_ERR_INVALID_ARG;
    *t = c->tune;
    return FF_OK;
}

ff_status ff_set_tuning(ff_context* c, const ff_tuning* t) {
    if (!c || !t) return FF_ERR_INVALID_ARG;
    if (t->radix_bits != 4 && t->radix_bits != 6 && t->radix_bits != 8) return FF_ERR_INVALID_ARG;
    if (t->sort_items != 4 && t->sort_items != 8 && t->sort_items != 16) return FF_ERR_INVALID_ARG;
    if (t->cells_block < 64 || t->cells_block > 1024 || (t->use_graph != 0 && t->use_graph != 1))
        return FF_ERR_INVALID_ARG;
    c->tune = *t;
    c->tune.cells_block = kBlock;   // the per-cell phase runs at the common block size
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
    char* stage = nullptr;
    ff_status st = begin_call(c, s, &stage);
    if (st != FF_OK) return st;
    Plan plan;
    std::string shape;
    st = build_desc(c, n_frames, frames, params, outs, stage, plan, shape);
    if (st != FF_OK) return st;
    const Ctx C = make_ctx(c);
    if (c->trace && (st = trace_collect(c)) != FF_OK) return st;
    if ((st = submit_desc(c, s, C, plan, batched)) != FF_OK) return st;
    if (batched && c->tune.use_graph && !c->trace) st = run_graph(c, C, plan, shape, s);
    else st = dispatch_plain(c, C, plan, s);
    if (st != FF_OK) return st;
    return end_call(c, s);
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

const char* ff_trace_slot_name(int32_t slot) {
    static const char* names[] = {"prep", "backproject_aabb", "coarse_hist", "coarse_scan_a",
                                  "coarse_scan_m", "coarse_scan_b", "keys", "cell_heads",
                                  "cells_top3_consistency_fuse", "final"};
    if (slot >= 0 && slot < 10) return names[slot];
    static const char* radix[] = {"radix_pass0", "radix_pass1", "radix_pass2", "radix_pass3",
                                  "radix_pass4", "radix_pass5", "radix_pass6", "radix_pass7",
                                  "radix_pass8", "radix_pass9", "radix_pass10", "radix_pass11",
                                  "radix_pass12", "radix_pass13", "radix_pass14", "radix_pass15"};
    if (slot >= 16 && slot < 32) return radix[slot - 16];
    return "unused";
}

ff_status ff_autotune(ff_context* c, int32_t n_frames, const ff_frame* frames,
                      const ff_params* params, const ff_output* outs, void* stream,
                      ff_tuning* chosen) {
    if (!c) return FF_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const ff_tuning keep = c->tune;
    ff_tuning best = keep;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    FF_HIP(hipEventCreate(&e0));
    FF_HIP(hipEventCreate(&e1));
    const int bits[] = {4, 6, 8};
    const int items[] = {4, 8, 16};
    ff_status st = FF_OK;
    for (int b : bits) {
        for (int it : items) {
            ff_tuning t = keep;
            t.radix_bits = b;
            t.sort_items = it;
            c->tune = t;
            if ((st = ff_fuse_batch(c, n_frames, frames, params, outs, stream)) != FF_OK) break;
            FF_HIP(hipEventRecord(e0, s));
            const int reps = 3;
            for (int r = 0; r < reps && st == FF_OK; ++r)
                st = ff_fuse_batch(c, n_frames, frames, params, outs, stream);
            FF_HIP(hipEventRecord(e1, s));
            FF_HIP(hipEventSynchronize(e1));
            float ms = 0;
            FF_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (st == FF_OK && ms < best_ms) { best_ms = ms; best = t; }
        }
        if (st != FF_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tune = (st == FF_OK) ? best : keep;
    if (chosen) *chosen = c->tune;
    return st;
}

}  // extern "C"
