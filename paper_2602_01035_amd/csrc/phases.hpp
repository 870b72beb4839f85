// Device phases of the fusion path for gfx950 (wave64, CDNA4).
//
// Each phase is a function of one work item (a tile of pixels, keys or cells).  The same
// functions run either as one kernel per phase (ff_fuse) or inside one persistent kernel
// that walks a global ticket space phase by phase (ff_fuse_batch).  Determinism: only
// integer atomics are used (histograms, counters); every floating-point reduction has a
// fixed order; compaction and sorting are stable, so members keep pixel-id order.
//
// Paper map: Eq. 8-9 -> backproject/gate; Sec. II.5(1) b-e -> AABB, coarse histogram,
// level selection, keys; the spatial hash grouping -> LSD radix sort of dense cell
// indices; Sec. II.5(2) a -> top-3 per cell; II.5(2) b and Eq. 4-7 -> view selection and
// consistency; Eq. 10-11 -> joint weight and fusion.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include "common.hpp"

namespace ff {

struct Ctx {
    const CallHdr* hdr;
    const DevFrame* frames;
    DevCam* cams;
    BatchState* bs;
    FrameState* fs;
    uint32_t* counts;        // [F][G^3] gated points per coarse cell
    uint64_t* fine_base;     // [F][G^3] first dense fine index of each coarse cell
    uint64_t* scan_tile;     // [n_scan_tiles] tile sums, then exclusive prefixes
    void* keysA;             // sort keys (u32 or u64 by BatchState::key64)
    void* keysB;
    uint32_t* valsA;         // batch pixel ids
    uint32_t* valsB;
    uint32_t* cell_start;    // [S + 1] first sorted position of each cell
    uint64_t* lb_tile;       // look-back words per tile (compactions)
    uint64_t* lb_digit;      // look-back words per (sort tile, digit)
    const uint32_t* epoch;
    uint32_t P_cap;          // entries of keys/vals/cell_start - 1
    uint32_t lb_tile_cap, lb_digit_cap;
};

// ---------------------------------------------------------------- small device helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t f2o(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float o2f(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every wait is bounded by wall-clock time (s_memrealtime ticks, limit in the call header)
// and gives up at once when another wait already gave up.
struct Waiter {
    uint64_t t0, limit;
    uint32_t n;
    __device__ __forceinline__ explicit Waiter(uint64_t lim) : t0(wall_clock64()), limit(lim), n(0) {}
    // true when the wait must stop
    __device__ __forceinline__ bool expired(BatchState* bs);
};

// true once any bounded wait has given up: every later wait returns at once, so a logic
// error can never turn into a long chain of timed-out waits
__device__ __forceinline__ bool aborted(BatchState* bs) {
    return ld_relaxed(&bs->error) & kErrSpin;
}
__device__ __forceinline__ bool Waiter::expired(BatchState* bs) {
    if ((++n & 31u) != 0) return false;
    return aborted(bs) || (wall_clock64() - t0) > limit;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ uint32_t wave_incl(uint32_t v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t n = __shfl_up(v, o);
        if (l >= (uint32_t)o) v += n;
    }
    return v;
}
__device__ __forceinline__ uint64_t wave_incl64(uint64_t v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t n = __shfl_up(v, o);
        if (l >= (uint32_t)o) v += n;
    }
    return v;
}

// Block-wide exclusive scan of one u32 per thread (256 threads); returns the block total.
__device__ __forceinline__ uint32_t block_excl(uint32_t v, uint32_t* s_w, uint32_t& total) {
    const uint32_t tid = threadIdx.x, w = tid / kWave, l = lane_id();
    uint32_t inc = wave_incl(v);
    if (l == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        uint32_t x = s_w[i];
        if ((uint32_t)i < w) off += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}
__device__ __forceinline__ uint64_t block_excl64(uint64_t v, uint64_t* s_w, uint64_t& total) {
    const uint32_t tid = threadIdx.x, w = tid / kWave, l = lane_id();
    uint64_t inc = wave_incl64(v);
    if (l == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        uint64_t x = s_w[i];
        if ((uint32_t)i < w) off += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

__device__ __forceinline__ void raise_error(BatchState* bs, uint32_t bit) {
    atomicOr(&bs->error, bit);
}

// Look-back word: high 32 bits = (tag << 2) | flag, low 32 bits = value.
// flag 1 = tile aggregate, 2 = inclusive prefix.
__device__ __forceinline__ uint64_t lb_word(uint32_t tag, uint32_t flag, uint32_t v) {
    return ((uint64_t)((tag << 2) | flag) << 32) | v;
}
__device__ __forceinline__ uint32_t lb_tag(uint32_t epoch, uint32_t slot) {
    return ((epoch << 5) | slot) & 0x3FFFFFFFu;
}

// Exclusive prefix of `tile` over earlier tiles (decoupled look-back, one wave, 64
// predecessors per step).  Every earlier tile was claimed by a running workgroup before
// this one (tickets), so each wait ends; a bounded spin guards against logic errors.
__device__ uint32_t lookback_wave(uint64_t* lb, uint32_t tile, uint32_t tag, BatchState* bs,
                                  uint64_t wait_ticks) {
    const uint32_t l = lane_id();
    Waiter wt(wait_ticks);
    uint32_t prefix = 0;
    int64_t base = (int64_t)tile - 1;
    while (base >= 0) {
        const int64_t idx = base - (int64_t)l;
        uint64_t w = 0;
        bool ready = idx < 0;
        while (true) {
            if (!ready) {
                w = ld_relaxed(&lb[idx]);
                const uint32_t hi = (uint32_t)(w >> 32);
                ready = ((hi >> 2) == tag) && (hi & 3u);
            }
            if (__all(ready)) break;
            if (wt.expired(bs)) {
                if (l == 0) raise_error(bs, kErrSpin);
                return prefix;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        const uint32_t hi = (uint32_t)(w >> 32);
        const uint32_t flag = idx < 0 ? 2u : (hi & 3u);
        const uint32_t val = idx < 0 ? 0u : (uint32_t)w;
        const uint64_t pm = __ballot(flag == 2u);
        const uint32_t first = pm ? (uint32_t)(__ffsll((unsigned long long)pm) - 1) : 64u;
        prefix += wave_sum(l <= first ? val : 0u);
        if (pm) break;
        base -= kWave;
    }
    return prefix;
}

// Single-thread look-back (one digit per thread in the radix passes).
__device__ uint32_t lookback_thread(uint64_t* lb, uint32_t tile, uint32_t stride, uint32_t d,
                                    uint32_t tag, BatchState* bs, uint64_t wait_ticks) {
    uint32_t prefix = 0;
    Waiter wt(wait_ticks);
    for (int64_t t = (int64_t)tile - 1; t >= 0; --t) {
        uint64_t w;
        uint32_t hi;
        while (true) {
            w = ld_relaxed(&lb[(uint64_t)t * stride + d]);
            hi = (uint32_t)(w >> 32);
            if (((hi >> 2) == tag) && (hi & 3u)) break;
            if (wt.expired(bs)) {
                raise_error(bs, kErrSpin);
                return prefix;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        prefix += (uint32_t)w;
        if ((hi & 3u) == 2u) break;
    }
    return prefix;
}

// ---------------------------------------------------------------- the method's arithmetic
// Canonical float32 order (no contraction: the library is built with -ffp-contract=off).

struct Pt {
    float x, y, z;
};

// Eq. 8: camera-frame point (d (x - cx)/fx, d (y - cy)/fy, d), then R^T X + c.
__device__ __forceinline__ Pt backproject(const DevCam& cm, float fxp, float fyp, float d) {
    const float xn = (fxp - cm.cx) / cm.fx;
    const float yn = (fyp - cm.cy) / cm.fy;
    const float X = xn * d, Y = yn * d, Z = d;
    Pt p;
    p.x = ((cm.R[0] * X + cm.R[3] * Y) + cm.R[6] * Z) + cm.c[0];
    p.y = ((cm.R[1] * X + cm.R[4] * Y) + cm.R[7] * Z) + cm.c[1];
    p.z = ((cm.R[2] * X + cm.R[5] * Y) + cm.R[8] * Z) + cm.c[2];
    return p;
}

// Eq. 9 (strict C > tau) plus a finite positive depth.
__device__ __forceinline__ bool gate_px(float d, float c, float tau, bool no_mf) {
    return __builtin_isfinite(d) && d > 0.0f && (no_mf || c > tau);
}
__device__ __forceinline__ bool finite3(const Pt& p) {
    return __builtin_isfinite(p.x) && __builtin_isfinite(p.y) && __builtin_isfinite(p.z);
}

// Eq. 4: nearest pixel of the projection into camera cm; false when behind or outside.
__device__ __forceinline__ bool project(const DevCam& cm, const Pt& p, int& px, int& py) {
    const float X = ((cm.R[0] * p.x + cm.R[1] * p.y) + cm.R[2] * p.z) + cm.t[0];
    const float Y = ((cm.R[3] * p.x + cm.R[4] * p.y) + cm.R[5] * p.z) + cm.t[1];
    const float Z = ((cm.R[6] * p.x + cm.R[7] * p.y) + cm.R[8] * p.z) + cm.t[2];
    const float u = cm.fx * (X / Z) + cm.cx;
    const float v = cm.fy * (Y / Z) + cm.cy;
    const float fu = floorf(u + 0.5f), fv = floorf(v + 0.5f);
    const bool ok = (Z > 0.0f) && (fu >= 0.0f) && (fu < (float)cm.W) && (fv >= 0.0f) &&
                    (fv < (float)cm.H);
    px = ok ? (int)fu : 0;
    py = ok ? (int)fv : 0;
    return ok;
}

// Sec. II.5(1)c: coarse edge 2^e, smallest power of two with G 2^e >= longest extent.
__device__ __forceinline__ int coarse_exponent(const float lo[3], const float hi[3], int log2G) {
    float ext = hi[0] - lo[0];
    const float e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
    if (e1 > ext) ext = e1;
    if (e2 > ext) ext = e2;
    if (ext == 0.0f) return kEMin;
    if (!__builtin_isfinite(ext)) return kEMax;
    const uint32_t b = __float_as_uint(ext);
    const int E = (int)((b >> 23) & 0xFFu);
    if (E == 0) return kEMin;                       // subnormal extent
    const int cl = (b & 0x7FFFFFu) ? (E - 126) : (E - 127);
    int e = cl - log2G;
    e = e < kEMin ? kEMin : e;
    e = e > kEMax ? kEMax : e;
    return e;
}

// Sec. II.5(1)d: the smallest level whose cells hold at most target * 4^L points.
__device__ __forceinline__ int level_of(uint32_t n, const DevParams& P) {
    if (P.level_override >= 0) return P.level_override;
    int L = 0;
    uint64_t cap = (uint64_t)P.target;
    while (L < P.Lmax && (uint64_t)n > cap) {
        ++L;
        cap <<= 2;
    }
    return L;
}

struct FrameGrid {
    float bmin[3];
    float scale;      // 2^-e
    int G, log2G;
};

__device__ __forceinline__ void frame_grid(const FrameState& st, const DevParams& P,
                                           FrameGrid& g) {
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = o2f(st.bmin_o[a]);
        hi[a] = o2f(st.bmax_o[a]);
        g.bmin[a] = lo[a];
    }
    const int e = coarse_exponent(lo, hi, P.log2G);
    g.scale = __uint_as_float((uint32_t)(127 - e) << 23);
    g.G = P.G;
    g.log2G = P.log2G;
}

struct CellCoord {
    float q[3];
    int ci[3];
    uint32_t lin;
};

__device__ __forceinline__ CellCoord coarse_cell(const FrameGrid& g, const Pt& p) {
    CellCoord c;
    const float pv[3] = {p.x, p.y, p.z};
    const float gm1 = (float)(g.G - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.q[a] = (pv[a] - g.bmin[a]) * g.scale;
        // q >= 0 for every point of the frame (bmin is their minimum); the lower clamp
        // only keeps a corrupted AABB from indexing outside the grid
        c.ci[a] = (int)fminf(fmaxf(floorf(c.q[a]), 0.0f), gm1);
    }
    c.lin = ((uint32_t)c.ci[2] * (uint32_t)g.G + (uint32_t)c.ci[1]) * (uint32_t)g.G +
            (uint32_t)c.ci[0];
    return c;
}

// Sec. II.5(1)e: local offsets inside the coarse cell at level L.
__device__ __forceinline__ void fine_local(const CellCoord& c, int L, int loc[3]) {
    const float s = (float)(1u << L);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float f = floorf(c.q[a] * s);
        f = fminf(f, (float)(c.ci[a] + 1) * s - 1.0f);
        loc[a] = (int)f - c.ci[a] * (1 << L);
    }
}

__device__ __forceinline__ uint64_t canonical_key(const CellCoord& c, const int loc[3],
                                                  int Lmax) {
    return ((uint64_t)c.lin << (3 * Lmax)) | ((uint64_t)loc[2] << (2 * Lmax)) |
           ((uint64_t)loc[1] << Lmax) | (uint64_t)loc[0];
}

// ---------------------------------------------------------------- lookups

// camera owning pixel tile `tile` (cams sorted by tile_off)
__device__ __forceinline__ int cam_of_tile(const Ctx& C, uint32_t tile) {
    int lo = 0, hi = (int)C.hdr->n_cams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (C.cams[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// camera owning batch pixel id (pix_off table staged in LDS)
__device__ __forceinline__ int cam_of_pix(const uint32_t* s_off, int n, uint32_t id) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= id) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- per-pixel tile walk

// Visit the 16 pixels of this thread in tile `tile` (4 groups of 4 consecutive pixels, the
// groups 1024 pixels apart, so that a wave reads 1 KiB contiguous per load).  f(g, j, x, y,
// d, c, in_range) is called in pixel order for each thread.
template <typename F>
__device__ __forceinline__ void for_tile_pixels(const DevCam& cm, uint32_t tile, F&& f) {
    const uint32_t npx = (uint32_t)cm.W * (uint32_t)cm.H;
    const uint32_t base = (tile - cm.tile_off) * (uint32_t)kPxTile;
    const uint32_t W = (uint32_t)cm.W;
#pragma unroll
    for (int g = 0; g < kPxPerThread / 4; ++g) {
        const uint32_t idx = base + (uint32_t)g * (kBlock * 4) + threadIdx.x * 4u;
        float d[4], c[4];
        if (cm.vec_ok && idx + 3 < npx) {
            const float4 dv = *reinterpret_cast<const float4*>(cm.depth + idx);
            const float4 cv = *reinterpret_cast<const float4*>(cm.conf + idx);
            d[0] = dv.x; d[1] = dv.y; d[2] = dv.z; d[3] = dv.w;
            c[0] = cv.x; c[1] = cv.y; c[2] = cv.z; c[3] = cv.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = idx + j < npx;
                d[j] = in ? cm.depth[idx + j] : 0.0f;
                c[j] = in ? cm.conf[idx + j] : 0.0f;
            }
        }
        uint32_t y = idx / W;
        uint32_t x = idx - y * W;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f(g, j, x, y, d[j], c[j], idx + j < npx, idx + j);
            if (++x == W) { x = 0; ++y; }
        }
    }
}

// ---------------------------------------------------------------- phase: back-project + AABB

__device__ void ph_backproject(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    const int ci = cam_of_tile(C, tile);
    const DevCam& cm = C.cams[ci];
    const bool no_mf = P.flags & 1u;
    uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u}, cnt = 0;
    for_tile_pixels(cm, tile, [&](int, int, uint32_t x, uint32_t y, float d, float c, bool in,
                                  uint32_t) {
        if (!in || !gate_px(d, c, P.tau, no_mf)) return;
        const Pt p = backproject(cm, (float)x, (float)y, d);
        if (!finite3(p)) return;
        const uint32_t o[3] = {f2o(p.x), f2o(p.y), f2o(p.z)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = o[a] < mn[a] ? o[a] : mn[a];
            mx[a] = o[a] > mx[a] ? o[a] : mx[a];
        }
        ++cnt;
    });
    // wave reduce, then one atomic per wave (integer, order-independent)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint32_t a1 = __shfl_xor(mn[a], o), a2 = __shfl_xor(mx[a], o);
            mn[a] = a1 < mn[a] ? a1 : mn[a];
            mx[a] = a2 > mx[a] ? a2 : mx[a];
        }
        cnt += __shfl_xor(cnt, o);
    }
    if (lane_id() == 0 && cnt) {
        FrameState& st = C.fs[cm.frame];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicMin(&st.bmin_o[a], mn[a]);
            atomicMax(&st.bmax_o[a], mx[a]);
        }
        atomicAdd(&st.M, cnt);
    }
}

// ---------------------------------------------------------------- phase: coarse histogram

__device__ void ph_hist(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    const int ci = cam_of_tile(C, tile);
    const DevCam& cm = C.cams[ci];
    const bool no_mf = P.flags & 1u;
    FrameGrid g;
    frame_grid(C.fs[cm.frame], P, g);
    uint32_t* counts = C.counts + (uint64_t)cm.frame * (uint64_t)(P.G * P.G * P.G);
    for_tile_pixels(cm, tile, [&](int, int, uint32_t x, uint32_t y, float d, float c, bool in,
                                  uint32_t) {
        bool has = in && gate_px(d, c, P.tau, no_mf);
        uint32_t key = 0;
        if (has) {
            const Pt p = backproject(cm, (float)x, (float)y, d);
            has = finite3(p);
            if (has) key = coarse_cell(g, p).lin;
        }
        // wavefront-level histogram: one atomic per distinct coarse cell in the wave
        uint64_t pending = __ballot(has);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const uint32_t lk = __shfl(key, leader);
            const uint64_t peers = __ballot(has && key == lk);
            if ((int)lane_id() == leader) atomicAdd(&counts[lk], (uint32_t)__popcll(peers));
            pending &= ~peers;
            if (key == lk) has = false;
        }
    });
}

// ---------------------------------------------------------------- phase: coarse scan
// span(c) = 8^L(c) dense fine indices for every occupied coarse cell; exclusive scan over
// (frame, cell) gives each cell's first dense index.  Three sub-phases: tile sums, a
// one-workgroup scan of the tile sums, and the per-tile scan.

__device__ __forceinline__ uint64_t span_of(uint32_t n, const DevParams& P) {
    return n ? (1ull << (3 * level_of(n, P))) : 0ull;
}

__device__ void ph_scan_a(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    const uint64_t total = (uint64_t)H.n_frames * (uint64_t)(P.G * P.G * P.G);
    uint64_t s = 0;
    const uint64_t base = (uint64_t)tile * kScanTile;
#pragma unroll 4
    for (int i = 0; i < kScanTile / kBlock; ++i) {
        const uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
        if (idx < total) s += span_of(C.counts[idx], P);
    }
    uint64_t* s_w = reinterpret_cast<uint64_t*>(smem);
    s = wave_sum64(s);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) C.scan_tile[tile] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__device__ void ph_scan_m(const Ctx& C, uint32_t, char* smem) {
    const CallHdr& H = *C.hdr;
    const uint32_t n = H.n_scan_tiles;
    uint64_t* s_w = reinterpret_cast<uint64_t*>(smem);
    uint64_t carry = 0;
    for (uint32_t b = 0; b < n; b += kBlock) {
        const uint32_t i = b + threadIdx.x;
        const uint64_t v = i < n ? C.scan_tile[i] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_excl64(v, s_w, tot);
        if (i < n) C.scan_tile[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        BatchState& bs = *C.bs;
        bs.T_tot = carry;
        const uint32_t bits = carry > 1 ? 64u - (uint32_t)__clzll((long long)(carry - 1)) : 0u;
        bs.key_bits = bits;
        bs.key64 = bits > 32 ? 1u : 0u;
        const uint32_t rb = H.radix_bits;
        uint32_t np = (bits + rb - 1) / rb;
        if (np > H.npass_max) {           // cannot happen: npass_max bounds the key width
            raise_error(C.bs, kErrBounds);
            np = H.npass_max;
        }
        bs.npass = np;
    }
}

__device__ void ph_scan_b(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    const uint64_t per_frame = (uint64_t)(P.G * P.G * P.G);
    const uint64_t total = (uint64_t)H.n_frames * per_frame;
    uint64_t* s_w = reinterpret_cast<uint64_t*>(smem);
    constexpr int kPer = kScanTile / kBlock;       // 16 consecutive cells per thread
    const uint64_t base = (uint64_t)tile * kScanTile + (uint64_t)threadIdx.x * kPer;
    uint64_t sp[kPer];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const uint64_t idx = base + i;
        sp[i] = idx < total ? span_of(C.counts[idx], P) : 0ull;
        s += sp[i];
    }
    uint64_t tot;
    uint64_t run = C.scan_tile[tile] + block_excl64(s, s_w, tot);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const uint64_t idx = base + i;
        if (idx < total) {
            C.fine_base[idx] = run;
            if (idx % per_frame == 0) C.fs[idx / per_frame].fine_begin = run;
        }
        run += sp[i];
    }
}

// ---------------------------------------------------------------- phase: keys + compaction

__device__ void ph_keys(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    BatchState* bs = C.bs;
    const int ci = cam_of_tile(C, tile);
    const DevCam& cm = C.cams[ci];
    const bool no_mf = P.flags & 1u;
    const bool no_sa = P.flags & 4u;
    const uint32_t G3 = (uint32_t)(P.G * P.G * P.G);
    const uint32_t* counts = C.counts + (uint64_t)cm.frame * G3;
    const uint64_t* fbase = C.fine_base + (uint64_t)cm.frame * G3;
    const bool key64 = bs->key64;
    const uint32_t npass = no_sa ? 0u : bs->npass;
    const uint32_t rb = H.radix_bits, D = 1u << rb;

    uint32_t* s_w = reinterpret_cast<uint32_t*>(smem);                 // [4]
    uint32_t* s_hist = s_w + 8;                                       // [npass][D]
    uint32_t* s_misc = s_hist + kMaxPass * kMaxDigits;                // [4]
    for (uint32_t i = threadIdx.x; i < npass * D; i += kBlock) s_hist[i] = 0;

    FrameGrid g;
    if (!no_sa) frame_grid(C.fs[cm.frame], P, g);

    uint64_t kv[kPxPerThread];
    uint32_t mask = 0;
    for_tile_pixels(cm, tile, [&](int gi, int j, uint32_t x, uint32_t y, float d, float c,
                                  bool in, uint32_t) {
        const int k = gi * 4 + j;
        kv[k] = 0;
        if (!in || !gate_px(d, c, P.tau, no_mf)) return;
        const Pt p = backproject(cm, (float)x, (float)y, d);
        if (!finite3(p)) return;
        mask |= 1u << k;
        if (no_sa) return;
        const CellCoord cc = coarse_cell(g, p);
        const int L = level_of(counts[cc.lin], P);
        int loc[3];
        fine_local(cc, L, loc);
        kv[k] = fbase[cc.lin] +
                ((((uint64_t)loc[2] << L) | (uint64_t)loc[1]) << L | (uint64_t)loc[0]);
    });
    __syncthreads();   // s_hist zeroed
    // per group of 4: exclusive ranks in pixel order (group-major, then thread, then j)
    uint32_t off[4], tile_total = 0;
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
        const uint32_t c = __popc((mask >> (gi * 4)) & 0xFu);
        uint32_t tot;
        off[gi] = tile_total + block_excl(c, s_w, tot);
        tile_total += tot;
    }
    // look-back for the tile's base position
    const uint32_t tag = lb_tag(*C.epoch, 0);
    if (threadIdx.x < kWave) {
        if (threadIdx.x == 0) st_relaxed(&C.lb_tile[tile], lb_word(tag, 1, tile_total));
        const uint32_t pre = lookback_wave(C.lb_tile, tile, tag, bs, H.wait_ticks);
        if (threadIdx.x == 0) {
            st_relaxed(&C.lb_tile[tile], lb_word(tag, 2, pre + tile_total));
            s_misc[0] = pre;
            if (tile == H.n_px_tiles - 1) bs->M_tot = pre + tile_total;
        }
    }
    __syncthreads();
    const uint32_t pre = s_misc[0];
    const uint32_t pbase = cm.pix_off + (tile - cm.tile_off) * (uint32_t)kPxTile;
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
        uint32_t o = pre + off[gi];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = gi * 4 + j;
            if (!(mask >> k & 1u)) continue;
            if (o >= C.P_cap) { raise_error(bs, kErrBounds); continue; }
            const uint32_t pid = pbase + (uint32_t)gi * (kBlock * 4) + threadIdx.x * 4u + j;
            if (key64) reinterpret_cast<uint64_t*>(C.keysA)[o] = kv[k];
            else reinterpret_cast<uint32_t*>(C.keysA)[o] = (uint32_t)kv[k];
            C.valsA[o] = pid;
            for (uint32_t ps = 0; ps < npass; ++ps)
                atomicAdd(&s_hist[ps * D + ((kv[k] >> (ps * rb)) & (D - 1))], 1u);
            ++o;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < npass * D; i += kBlock) {
        const uint32_t v = s_hist[i];
        if (v) atomicAdd(&bs->digit_hist[i / D][i % D], v);
    }
}

// ---------------------------------------------------------------- phase: one LSD radix pass
// Onesweep-style: stable rank inside the tile by wave-level digit matching, per-digit
// decoupled look-back across tiles, LDS staging so that writes go out in digit runs.

template <typename K, int ITEMS>
__device__ void radix_pass(const Ctx& C, uint32_t pass, uint32_t tile, char* smem) {
    constexpr int KT = kBlock * ITEMS;
    const CallHdr& H = *C.hdr;
    BatchState* bs = C.bs;
    const uint32_t n = min(bs->M_tot, C.P_cap);
    const uint32_t rb = H.radix_bits, D = 1u << rb;
    const uint32_t shift = pass * rb;
    if ((uint64_t)tile * KT >= n) return;
    const K* kin = reinterpret_cast<const K*>((pass & 1) ? C.keysB : C.keysA);
    const uint32_t* vin = (pass & 1) ? C.valsB : C.valsA;
    K* kout = reinterpret_cast<K*>((pass & 1) ? C.keysA : C.keysB);
    uint32_t* vout = (pass & 1) ? C.valsA : C.valsB;

    K* s_key = reinterpret_cast<K*>(smem);                              // [KT]
    uint32_t* s_val = reinterpret_cast<uint32_t*>(s_key + KT);          // [KT]
    uint32_t* s_wc = s_val + KT;                                        // [4][D] per-wave counts
    uint32_t* s_doff = s_wc + 4 * kMaxDigits;                           // [D] tile digit offsets
    uint32_t* s_gb = s_doff + kMaxDigits;                               // [D] global base
    uint32_t* s_w = s_gb + kMaxDigits;                                  // [8]
    const uint32_t tid = threadIdx.x, w = tid / kWave, l = lane_id();
    for (uint32_t i = tid; i < 4 * D; i += kBlock) s_wc[i] = 0;
    __syncthreads();

    // load (wave-striped: wave w owns a contiguous run of ITEMS*64 keys)
    const uint64_t t0 = (uint64_t)tile * KT + (uint64_t)w * (ITEMS * kWave);
    K key[ITEMS];
    uint32_t val[ITEMS], rank[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint64_t idx = t0 + (uint64_t)i * kWave + l;
        const bool in = idx < n;
        key[i] = in ? kin[idx] : (K)0;
        val[i] = in ? vin[idx] : 0u;
    }
    const uint64_t lt = (l == 0) ? 0ull : ((~0ull) >> (64 - l));
    uint32_t* wc = s_wc + w * D;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint64_t idx = t0 + (uint64_t)i * kWave + l;
        const bool in = idx < n;
        const uint32_t dg = (uint32_t)(key[i] >> shift) & (D - 1);
        uint64_t peers = __ballot(in);
        for (uint32_t b = 0; b < rb; ++b) {
            const uint64_t bal = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t before = wc[dg];
        const uint32_t lower = (uint32_t)__popcll(peers & lt);
        rank[i] = before + lower;
        // the lowest lane of each peer group bumps the counter after everyone has read it
        __builtin_amdgcn_wave_barrier();
        if (in && lower == 0) wc[dg] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per-digit tile totals and per-wave offsets
    uint32_t dtot = 0;
    if (tid < D) {
        uint32_t acc = 0;
        for (int ww = 0; ww < 4; ++ww) {
            const uint32_t c = s_wc[ww * D + tid];
            s_wc[ww * D + tid] = acc;
            acc += c;
        }
        dtot = acc;
    }
    const uint32_t tag = lb_tag(*C.epoch, 2 + pass);
    uint64_t* lb = C.lb_digit;
    if (tid < D) st_relaxed(&lb[(uint64_t)tile * D + tid], lb_word(tag, 1, dtot));
    uint32_t tot_unused;
    const uint32_t doff = block_excl(tid < D ? dtot : 0u, s_w, tot_unused);
    if (tid < D) s_doff[tid] = doff;
    __syncthreads();
    // scatter into LDS in (digit, original order)
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint64_t idx = t0 + (uint64_t)i * kWave + l;
        if (idx >= n) continue;
        const uint32_t dg = (uint32_t)(key[i] >> shift) & (D - 1);
        const uint32_t pos = s_doff[dg] + s_wc[w * D + dg] + rank[i];
        s_key[pos] = key[i];
        s_val[pos] = val[i];
    }
    // global base of each digit: digit start + prefix of earlier tiles
    const uint32_t dstart = block_excl(tid < D ? bs->digit_hist[pass][tid] : 0u, s_w, tot_unused);
    if (tid < D) {
        const uint32_t pre = lookback_thread(lb, tile, D, tid, tag, bs, H.wait_ticks);
        st_relaxed(&lb[(uint64_t)tile * D + tid], lb_word(tag, 2, pre + dtot));
        s_gb[tid] = dstart + pre - s_doff[tid];
    }
    __syncthreads();
    const uint32_t cnt = (uint32_t)((n - (uint64_t)tile * KT) < (uint64_t)KT
                                        ? (n - (uint64_t)tile * KT) : (uint64_t)KT);
    for (uint32_t s = tid; s < cnt; s += kBlock) {
        const K kk = s_key[s];
        const uint32_t dg = (uint32_t)(kk >> shift) & (D - 1);
        const uint32_t dst = s_gb[dg] + s;
        if (dst >= n) { raise_error(bs, kErrBounds); continue; }
        kout[dst] = kk;
        vout[dst] = s_val[s];
    }
}

template <int ITEMS>
__device__ void ph_radix(const Ctx& C, uint32_t pass, uint32_t tile, char* smem) {
    BatchState* bs = C.bs;
    if (C.hdr->prm.flags & 4u) return;
    if (pass >= bs->npass) return;
    if (bs->key64) radix_pass<uint64_t, ITEMS>(C, pass, tile, smem);
    else radix_pass<uint32_t, ITEMS>(C, pass, tile, smem);
}

// final (sorted) buffers
__device__ __forceinline__ const uint32_t* sorted_vals(const Ctx& C) {
    return (C.bs->npass & 1) ? C.valsB : C.valsA;
}
__device__ __forceinline__ uint64_t sorted_key(const Ctx& C, uint32_t i) {
    const bool b = C.bs->npass & 1;
    if (C.bs->key64) return reinterpret_cast<const uint64_t*>(b ? C.keysB : C.keysA)[i];
    return reinterpret_cast<const uint32_t*>(b ? C.keysB : C.keysA)[i];
}

// frame index of a batch pixel id (frames staged in LDS by pix_begin)
__device__ __forceinline__ int frame_of_pix(const uint32_t* s_fpix, int nf, uint32_t id) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_fpix[mid] <= id) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- phase: cell heads

template <int ITEMS>
__device__ void ph_heads(const Ctx& C, uint32_t tile, char* smem) {
    constexpr int KT = kBlock * ITEMS;
    const CallHdr& H = *C.hdr;
    BatchState* bs = C.bs;
    if (H.prm.flags & 4u) return;
    const uint32_t n = min(bs->M_tot, C.P_cap);
    const uint32_t tag = lb_tag(*C.epoch, 1);
    uint32_t* s_w = reinterpret_cast<uint32_t*>(smem);        // [8]
    uint32_t* s_fpix = s_w + 8;                               // [F]
    uint32_t* s_fcnt = s_fpix + 64;                           // [F]
    const uint32_t nf = H.n_frames;
    for (uint32_t f = threadIdx.x; f < nf; f += kBlock) {
        s_fpix[f] = C.frames[f].pix_begin;
        s_fcnt[f] = 0;
    }
    __syncthreads();
    const uint64_t t0 = (uint64_t)tile * KT + (uint64_t)threadIdx.x * ITEMS;
    const bool active = (uint64_t)tile * KT < n;
    // thread-contiguous items so that the compaction keeps order
    uint32_t hmask = 0, c = 0;
    uint64_t prev = 0;
    if (active) {
        for (int i = 0; i < ITEMS; ++i) {
            const uint64_t idx = t0 + i;
            if (idx >= n) break;
            const uint64_t k = sorted_key(C, (uint32_t)idx);
            if (i == 0) prev = idx ? sorted_key(C, (uint32_t)idx - 1) : ~k;
            if (idx == 0 || k != prev) { hmask |= 1u << i; ++c; }
            prev = k;
        }
    }
    uint32_t tot;
    const uint32_t ex = block_excl(c, s_w, tot);
    __shared__ uint32_t s_pre;
    if (threadIdx.x < kWave) {
        if (active) {
            if (threadIdx.x == 0) st_relaxed(&C.lb_tile[tile], lb_word(tag, 1, tot));
            const uint32_t pre = lookback_wave(C.lb_tile, tile, tag, bs, H.wait_ticks);
            if (threadIdx.x == 0) {
                st_relaxed(&C.lb_tile[tile], lb_word(tag, 2, pre + tot));
                s_pre = pre;
                if ((uint64_t)(tile + 1) * KT >= n) {   // last real tile
                    bs->S_tot = pre + tot;
                    if (pre + tot <= C.P_cap) C.cell_start[pre + tot] = n;
                }
            }
        }
    }
    __syncthreads();
    if (!active) return;
    uint32_t o = s_pre + ex;
    const uint32_t* vals = sorted_vals(C);
    for (int i = 0; i < ITEMS; ++i) {
        if (!(hmask >> i & 1u)) continue;
        const uint32_t idx = (uint32_t)(t0 + i);
        if (o < C.P_cap) C.cell_start[o] = idx; else raise_error(bs, kErrBounds);
        ++o;
        const int f = frame_of_pix(s_fpix, (int)nf, vals[idx]);
        atomicAdd(&s_fcnt[f], 1u);
    }
    __syncthreads();
    for (uint32_t f = threadIdx.x; f < nf; f += kBlock)
        if (s_fcnt[f]) atomicAdd(&C.fs[f].S, s_fcnt[f]);
}

// ---------------------------------------------------------------- phase: cells
// One thread per cell: top-3 representatives (Sec. II.5(2)a), local views and
// consistency (II.5(2)b, Eq. 4-7), joint weight and fusion (Eq. 10-11), output.

struct Cand {
    float C;
    uint32_t id;     // batch pixel id
    int cam;
    bool hasp;
    Pt p;
};

struct CellsShared {
    uint32_t cam_pix[kMaxBatchCams];            // batch pix_off per camera (sorted)
    uint32_t fpix[kMaxFrames];                  // frame pix_begin
    uint32_t key_begin[kMaxFrames];             // frame's first sorted/compacted position
    uint32_t cell_begin[kMaxFrames];            // frame's first global cell
};

__device__ __forceinline__ void ensure_p(const Ctx& C, Cand& a) {
    if (a.hasp) return;
    const DevCam& cm = C.cams[a.cam];
    const uint32_t loc = a.id - cm.pix_off;
    const uint32_t y = loc / (uint32_t)cm.W, x = loc - y * (uint32_t)cm.W;
    a.p = backproject(cm, (float)x, (float)y, cm.depth[loc]);
    a.hasp = true;
}

// strict "a ranks before b": C descending, then x, y, z ascending, then pixel id
__device__ __forceinline__ bool rank_before(const Ctx& C, Cand& a, Cand& b) {
    if (a.C != b.C) return a.C > b.C;
    ensure_p(C, a);
    ensure_p(C, b);
    if (a.p.x != b.p.x) return a.p.x < b.p.x;
    if (a.p.y != b.p.y) return a.p.y < b.p.y;
    if (a.p.z != b.p.z) return a.p.z < b.p.z;
    return a.id < b.id;
}

// -ln V of representative (cam ri, point p): Eq. 4-7 over the first K-1 views by distance
__device__ double neg_log_v(const Ctx& C, int ri, const Pt& p, uint32_t fcam0, uint32_t fcams,
                            const DevParams& P) {
    const int keep = (P.K < (int)fcams ? P.K : (int)fcams) - 1;
    if (keep <= 0) return 0.0;
    float bd[kMaxK - 1];
    uint32_t br[kMaxK - 1];
    int bj[kMaxK - 1], bx[kMaxK - 1], by[kMaxK - 1];
    int nb = 0;
    for (uint32_t j = fcam0; j < fcam0 + fcams; ++j) {
        if ((int)j == ri) continue;
        const DevCam& cj = C.cams[j];
        int px, py;
        if (!project(cj, p, px, py)) continue;
        const float dx = p.x - cj.c[0], dy = p.y - cj.c[1], dz = p.z - cj.c[2];
        const float d2 = (dx * dx + dy * dy) + dz * dz;
        // insertion into the sorted list of the best `keep` candidates: carry the
        // candidate down the list, swapping with every entry it ranks before (slots past
        // nb are free, so whatever is carried into them is discarded)
        float cd = d2;
        uint32_t cr = cj.rank;
        int cjx = (int)j, cx = px, cy = py;
#pragma unroll
        for (int q = 0; q < kMaxK - 1; ++q) {
            if (q < keep && (q >= nb || cd < bd[q] || (cd == bd[q] && cr < br[q]))) {
                const float td = bd[q]; bd[q] = cd; cd = td;
                const uint32_t tr = br[q]; br[q] = cr; cr = tr;
                const int tj = bj[q]; bj[q] = cjx; cjx = tj;
                const int tx = bx[q]; bx[q] = cx; cx = tx;
                const int ty = by[q]; by[q] = cy; cy = ty;
            }
        }
        if (nb < keep) ++nb;
    }
    double s = 0.0;
    int m = 0;
#pragma unroll
    for (int q = 0; q < kMaxK - 1; ++q) {
        if (q >= nb) continue;
        const DevCam& cj = C.cams[bj[q]];
        const float d = cj.depth[(uint32_t)by[q] * (uint32_t)cj.W + (uint32_t)bx[q]];
        if (!(__builtin_isfinite(d) && d > 0.0f)) continue;
        const Pt Q = backproject(cj, (float)bx[q], (float)by[q], d);
        const double ex = (double)p.x - (double)Q.x;
        const double ey = (double)p.y - (double)Q.y;
        const double ez = (double)p.z - (double)Q.z;
        s += (ex * ex + ey * ey) + ez * ez;
        ++m;
    }
    if (m == 0) return 0.0;
    const double sig = (double)P.sigma;
    return s / ((double)m * (sig * sig));
}

__device__ void emit_cell(const Ctx& C, const DevFrame& fr, uint32_t o, Cand* rep, int nrep,
                          const double* expo, uint32_t nmem, uint64_t key) {
    double a[3] = {0.0, 0.0, 0.0}, amax = -INFINITY;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        if (r >= nrep) continue;
        a[r] = log((double)rep[r].C) - expo[r];
        amax = a[r] > amax ? a[r] : amax;
    }
    double ex[3] = {0.0, 0.0, 0.0};
    double se = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        if (r < nrep) ex[r] = exp(a[r] - amax);
        se += ex[r];
    }
    double x = 0.0, y = 0.0, z = 0.0, wsum = 0.0;
    double cr = 0.0, cg = 0.0, cb = 0.0;
    const bool rgb = fr.rgb != nullptr && fr.has_rgb;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double pi = ex[r] / se;
        if (r < nrep) {
            x += pi * (double)rep[r].p.x;
            y += pi * (double)rep[r].p.y;
            z += pi * (double)rep[r].p.z;
            wsum += (double)rep[r].C * exp(-expo[r]);
            if (rgb) {
                const DevCam& cm = C.cams[rep[r].cam];
                const uint8_t* px = cm.rgb + (uint64_t)(rep[r].id - cm.pix_off) * 3;
                cr += pi * (double)px[0];
                cg += pi * (double)px[1];
                cb += pi * (double)px[2];
            }
        } else {
            x += pi * 0.0; y += pi * 0.0; z += pi * 0.0;
            wsum += 0.0;
        }
    }
    fr.xyz[(uint64_t)o * 3 + 0] = (float)x;
    fr.xyz[(uint64_t)o * 3 + 1] = (float)y;
    fr.xyz[(uint64_t)o * 3 + 2] = (float)z;
    fr.weight[o] = (float)(wsum / (double)nrep);
    if (rgb) {
        const double v[3] = {cr, cg, cb};
        for (int k = 0; k < 3; ++k) {
            double t = rint(v[k]);
            t = t < 0.0 ? 0.0 : (t > 255.0 ? 255.0 : t);
            fr.rgb[(uint64_t)o * 3 + k] = (uint8_t)t;
        }
    }
    if (fr.n_members) fr.n_members[o] = nmem;
    if (fr.reps) {
        for (int r = 0; r < 3; ++r)
            fr.reps[(uint64_t)o * 3 + r] = r < nrep ? rep[r].id - fr.pix_begin : kPad;
    }
    if (fr.keys) fr.keys[o] = key;
}

__device__ void ph_cells(const Ctx& C, uint32_t item, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    BatchState* bs = C.bs;
    CellsShared& sh = *reinterpret_cast<CellsShared*>(smem);
    const uint32_t nf = H.n_frames, nc = H.n_cams;
    const bool no_sa = P.flags & 4u, no_mf = P.flags & 1u, no_dc = P.flags & 2u;
    for (uint32_t i = threadIdx.x; i < nc; i += kBlock) sh.cam_pix[i] = C.cams[i].pix_off;
    if (threadIdx.x == 0) {
        uint32_t kb = 0, cb = 0;
        for (uint32_t f = 0; f < nf; ++f) {
            sh.fpix[f] = C.frames[f].pix_begin;
            sh.key_begin[f] = kb;
            sh.cell_begin[f] = cb;
            kb += C.fs[f].M;
            cb += no_sa ? C.fs[f].M : C.fs[f].S;
        }
    }
    __syncthreads();
    const uint32_t M_tot = min(bs->M_tot, C.P_cap);
    const uint32_t S = min(no_sa ? bs->M_tot : bs->S_tot, M_tot);
    const uint32_t n_items = H.n_cell_items;
    const uint32_t b0 = (uint32_t)(((uint64_t)S * item) / n_items);
    const uint32_t b1 = (uint32_t)(((uint64_t)S * (item + 1)) / n_items);
    const uint32_t* vals = no_sa ? C.valsA : sorted_vals(C);
    const uint32_t G3 = (uint32_t)(P.G * P.G * P.G);
    uint32_t rsum_frame = 0xFFFFFFFFu, rsum = 0;
    for (uint32_t s = b0 + threadIdx.x; s < b1; s += kBlock) {
        uint32_t start, end;
        if (no_sa) { start = s; end = s + 1; }
        else { start = C.cell_start[s]; end = C.cell_start[s + 1]; }
        if (end > M_tot || start >= end) { raise_error(bs, kErrBounds); continue; }
        const uint32_t id0 = vals[start];
        const int f = frame_of_pix(sh.fpix, (int)nf, id0);
        if (id0 >= H.P_tot) { raise_error(bs, kErrBounds); continue; }
        const DevFrame& fr = C.frames[f];
        Cand rep[3];
        int nrep = 0;
        for (uint32_t k = start; k < end; ++k) {
            Cand c;
            c.id = vals[k];
            c.cam = cam_of_pix(sh.cam_pix, (int)nc, c.id);
            const DevCam& cm = C.cams[c.cam];
            if (c.id - cm.pix_off >= (uint32_t)cm.W * (uint32_t)cm.H) {
                raise_error(bs, kErrBounds);
                continue;
            }
            c.C = no_mf ? 1.0f : cm.conf[c.id - cm.pix_off];
            c.hasp = false;
            if (nrep == 3 && !rank_before(C, c, rep[2])) continue;
            if (nrep < 1 || rank_before(C, c, rep[0])) {
                rep[2] = rep[1]; rep[1] = rep[0]; rep[0] = c;
            } else if (nrep < 2 || rank_before(C, c, rep[1])) {
                rep[2] = rep[1]; rep[1] = c;
            } else {
                rep[2] = c;
            }
            if (nrep < 3) ++nrep;
        }
        double expo[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (r >= nrep) continue;
            ensure_p(C, rep[r]);
            if (!no_dc) expo[r] = neg_log_v(C, rep[r].cam, rep[r].p, fr.cam_begin, fr.n_cams, P);
        }
        uint64_t key;
        if (no_sa) {
            key = rep[0].id - fr.pix_begin;
        } else {
            FrameGrid g;
            frame_grid(C.fs[f], P, g);
            const CellCoord cc = coarse_cell(g, rep[0].p);
            const int L = level_of(C.counts[(uint64_t)f * G3 + cc.lin], P);
            int loc[3];
            fine_local(cc, L, loc);
            key = canonical_key(cc, loc, P.Lmax);
        }
        const uint32_t o = s - sh.cell_begin[f];
        if (o < fr.capacity) {
            emit_cell(C, fr, o, rep, nrep, expo, end - start, key);
            if (fr.moff) fr.moff[o] = start - sh.key_begin[f];
        }
        if (fr.mids) {
            for (uint32_t k = start; k < end; ++k) {
                const uint32_t mo = k - sh.key_begin[f];
                if (mo < fr.member_capacity) fr.mids[mo] = vals[k] - fr.pix_begin;
            }
        }
        // representatives per frame (aggregated per thread run, flushed on frame change)
        if ((uint32_t)f != rsum_frame) {
            if (rsum) atomicAdd(&C.fs[rsum_frame].R, rsum);
            rsum_frame = (uint32_t)f;
            rsum = 0;
        }
        rsum += (uint32_t)nrep;
    }
    if (rsum) atomicAdd(&C.fs[rsum_frame].R, rsum);
}

// ---------------------------------------------------------------- phase: final counts

__device__ void ph_final(const Ctx& C, uint32_t, char*) {
    const CallHdr& H = *C.hdr;
    const bool no_sa = H.prm.flags & 4u;
    for (uint32_t f = threadIdx.x; f < H.n_frames; f += kBlock) {
        const DevFrame& fr = C.frames[f];
        const FrameState& st = C.fs[f];
        const uint32_t S = no_sa ? st.M : st.S;
        if (fr.moff && S <= fr.capacity) fr.moff[S] = st.M;
        *fr.count = S;
        *fr.status = (S > fr.capacity || (fr.mids && st.M > fr.member_capacity))
                         ? 1 : (C.bs->error ? 2 : 0);
        if (fr.info) {
            fr.info[0] = st.M;
            fr.info[1] = S;
            fr.info[2] = st.R;
            fr.info[3] = C.bs->key_bits;
        }
    }
}

}  // namespace ff
