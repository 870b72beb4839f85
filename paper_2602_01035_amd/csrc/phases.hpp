// Device phases of the fusion path for gfx950 (wave64, CDNA4).
//
// Each phase is a function of one work item (a tile of pixels, keys or cells); the host
// launches one kernel per phase with one workgroup per item.  Design rules for MI355X:
//  * no same-address global atomics (they serialise at the memory side): per-tile partials
//    are written with plain stores and reduced by a small phase;
//  * no decoupled look-back (each step would be a coherent cross-XCD load of ~1-2 us):
//    compactions and the radix sort use counts + scan + scatter;
//  * only integer atomics, so every result is deterministic; compaction and the LSD radix
//    sort are stable, so the members of a cell keep pixel-id order.
//
// Paper map: Eq. 8-9 -> backproject / gate; Sec. II.5(1) b-e -> extents, coarse density,
// level selection, cell keys; the spatial hash grouping -> LSD radix sort of dense cell
// indices + segment heads; Sec. II.5(2) a -> top-3 per cell; II.5(2) b and Eq. 4-7 -> view
// selection and distance consistency; Eq. 10-11 -> joint weight and fusion.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include "common.hpp"

namespace ff {

struct Ctx {
    const CallHdr* hdr;
    const DevFrame* frames;
    const uint16_t* tile_cam;       // camera of every pixel tile
    DevCam* cams;
    BatchState* bs;
    FrameState* fs;
    TilePart* tiles;         // [n_px_tiles] AABB partials and gated counts
    uint32_t* tile_off;      // [n_px_tiles] first compacted position of each pixel tile
    uint32_t* counts;        // [F][G^3] gated points per coarse cell
    uint64_t* fine_base;     // [F][G^3] first dense fine index of each coarse cell
    uint8_t* level;          // [F][G^3] refinement level of each coarse cell
    CamClass* cls;           // [F][G^3] field-of-view class of the frame's cameras (occupied cells)
    uint64_t* scan_tile;     // [n_scan_tiles] tile sums, then exclusive prefixes
    void* keysA;             // sort keys (u32 or u64 by BatchState::key64)
    void* keysB;
    uint32_t* valsA;         // batch pixel ids
    uint32_t* valsB;
    uint32_t* digit_hist;    // [kMaxDigits][n_sort_tiles] per-tile digit counts / offsets
    uint32_t* digit_total;   // [kMaxDigits]
    uint32_t* head_cnt;      // [n_sort_tiles] cell heads per sort tile, then offsets
    uint32_t* cell_start;    // [S + 1] first sorted position of each cell
    uint32_t* conf_sorted;   // [M] confidence bits of each key in sorted order
    CamLite* camlite;        // [n_cams]
    float* raytab;           // per camera: (x - cx)/fx for each column, (y - cy)/fy per row
    uint32_t P_cap;          // entries of keys/vals (cell_start has P_cap + 2)
    uint32_t sort_tiles_cap;
};

// ---------------------------------------------------------------- small device helpers

// Pointers read out of descriptors are generic to the compiler: accessed as such they
// compile to flat instructions, which also count against the LDS wait counter and so
// serialise LDS reads behind outstanding global loads.  Every descriptor pointer refers to
// device global memory, which glob() states.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* glob(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t f2o(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float o2f(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
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
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* s_w) {
    uint32_t tot;
    (void)block_excl(v, s_w, tot);
    return tot;
}

__device__ __forceinline__ void raise_error(BatchState* bs, uint32_t bit) {
    atomicOr(&bs->error, bit);
}

// Lanes of the wave holding the same value `d` among the active ones of `valid`, using
// one ballot per bit of a `bits`-wide value.
__device__ __forceinline__ uint64_t match_peers(uint32_t d, bool valid, uint32_t bits) {
    uint64_t peers = __ballot(valid);
    for (uint32_t b = 0; b < bits; ++b) {
        // m: all ones where bit b of d is set; lanes that agree on the bit are those where
        // the ballot equals m
        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)d, (int)b, 1);
        const uint64_t bal = __ballot(m != 0u);
        peers &= ~(bal ^ ((uint64_t)m << 32 | m));
    }
    return peers;
}

// ---------------------------------------------------------------- the method's arithmetic
// Canonical float32 order (no contraction: the library is built with -ffp-contract=off).

struct Pt {
    float x, y, z;
};

// Eq. 8: camera-frame point (d (x - cx)/fx, d (y - cy)/fy, d), then R^T X + c.
// The same with the normalised ray (xn, yn) = ((x - cx)/fx, (y - cy)/fy) already divided
// out (per-camera tables hold exactly these float32 quotients).
template <typename Cam>
__device__ __forceinline__ Pt backproject_ray(const Cam& cm, float xn, float yn, float d) {
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

// Eq. 4 field-of-view decision: camera-frame point X = R p + t, in front (Z > 0), and the
// nearest pixel floor(u + 1/2), floor(v + 1/2) of u = fx X/Z + cx, v = fy Y/Z + cy inside
// the image.  The division is done only where it matters: an approximate reciprocal decides
// points clearly inside or outside, and the exact IEEE quotients decide points near a
// border.  The approximate u + 1/2 (one fused multiply-add onto cx + 1/2) differs from the
// exact one by at most 3.6e-7 |fx X/Z| plus two half-ulps of the sums; with the camera
// range the boundary admits (sides and principal point within 2^14 px) that is < 0.04 px
// wherever |u| < 2^16, inside the 1/16 px margin, and beyond 2^16 the point is outside by
// far more than the error.  The ranges are tested as med3(t, lo, hi) == t, which holds
// exactly when lo <= t <= hi and never for a NaN t; the upper ends are the largest floats
// below W - m (clearly inside) and W + m (not clearly outside), so the tests are the
// half-open intervals.  The bound needs an accurate reciprocal, so unless the approximate
// reciprocal is a positive normal float (a subnormal Z has an infinite one, and X times it
// may be infinite while X/Z is small; above 2^126 the reciprocal is subnormal and may be
// flushed to 0) the point is never clearly anything, and neither is an approximation that
// is not a number; both go to the exact quotients.  Written without early exits: only the
// rare border case branches.
constexpr float kFovMargin = 0.0625f;
template <typename Cam>
__device__ __forceinline__ bool in_view_fast(const Cam& cm, const Pt& p) {
    const float Z = ((cm.R[6] * p.x + cm.R[7] * p.y) + cm.R[8] * p.z) + cm.t[2];
    const float X = ((cm.R[0] * p.x + cm.R[1] * p.y) + cm.R[2] * p.z) + cm.t[0];
    const float Y = ((cm.R[3] * p.x + cm.R[4] * p.y) + cm.R[5] * p.z) + cm.t[1];
    const float rz = __builtin_amdgcn_rcpf(Z);
    const float ta = __builtin_fmaf(cm.fx, X * rz, cm.cxh);
    const float tb = __builtin_fmaf(cm.fy, Y * rz, cm.cyh);
    const float m = kFovMargin;
    const bool front = Z > 0.0f;
    // the approximate reciprocal is a positive normal float: Z > 0, not subnormal (whose
    // reciprocal is infinite or flushed) and below 2^126 (whose reciprocal is subnormal)
    const bool normal_z = __builtin_amdgcn_classf(rz, 1 << 8);
    const bool sure_in = normal_z & (__builtin_amdgcn_fmed3f(ta, m, cm.in_hx) == ta) &
                         (__builtin_amdgcn_fmed3f(tb, m, cm.in_hy) == tb);
    const bool near = (__builtin_amdgcn_fmed3f(ta, -m, cm.out_hx) == ta) &
                      (__builtin_amdgcn_fmed3f(tb, -m, cm.out_hy) == tb);
    const bool sure_out = normal_z & !near & !__builtin_isunordered(ta, tb);
    bool in = front & sure_in;
    if (front & !sure_in & !sure_out) {
        const float W = (float)cm.W, H = (float)cm.H;
        const float u = cm.fx * (X / Z) + cm.cx, v = cm.fy * (Y / Z) + cm.cy;
        const float fu = floorf(u + 0.5f), fv = floorf(v + 0.5f);
        in = (fu >= 0.0f) && (fu < W) && (fv >= 0.0f) && (fv < H);
    }
    return in;
}

// the largest float below a positive finite x
__device__ __forceinline__ float float_below(float x) {
    return __uint_as_float(__float_as_uint(x) - 1u);
}

// exact nearest pixel of a point known to be in view (the arithmetic of the exact branch
// of in_view_fast)
template <typename Cam>
__device__ __forceinline__ void exact_pixel(const Cam& cm, float X, float Y, float Z, int& px,
                                            int& py) {
    const float u = cm.fx * (X / Z) + cm.cx, v = cm.fy * (Y / Z) + cm.cy;
    px = (int)floorf(u + 0.5f);
    py = (int)floorf(v + 0.5f);
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
    int G;
};

__device__ __forceinline__ void frame_grid(const FrameState& st, const DevParams& P,
                                           FrameGrid& g) {
#pragma unroll
    for (int a = 0; a < 3; ++a) g.bmin[a] = st.bmin[a];
    g.scale = st.scale;
    g.G = P.G;
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

// camera owning pixel tile `tile` (a table the host writes with the descriptor)
__device__ __forceinline__ int cam_of_tile(const Ctx& C, uint32_t tile) {
    return (int)C.tile_cam[tile];
}

// index of the last entry <= id in an ascending table (camera or frame pixel offsets)
__device__ __forceinline__ int last_le(const uint32_t* tab, int n, uint32_t id) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid] <= id) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// camera centre c = -R^T t in the canonical order (Eq. 8's inverse extrinsics)
__device__ __forceinline__ void camera_centre(DevCam& cm) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
        cm.c[a] = -((cm.R[0 * 3 + a] * cm.t[0] + cm.R[1 * 3 + a] * cm.t[1]) +
                    cm.R[2 * 3 + a] * cm.t[2]);
}

// ---------------------------------------------------------------- per-pixel tile walk

// A pixel tile is 4096 pixels of one camera, 16 per thread: 4 groups of 4 consecutive
// pixels, the groups 1024 pixels apart, so that a wave reads 1 KiB contiguous per load.
// Thread t holds pixels base + g * 1024 + 4 t + j (g < 4, j < 4), loaded as float4 where
// aligned.
struct TileData {
    float d[kPxPerThread / 4][4], c[kPxPerThread / 4][4];
};

// every load of the thread (16 depths and 16 confidences in flight)
__device__ __forceinline__ void load_tile(const DevCam& cm, uint32_t tile, TileData& t) {
    const uint32_t npx = (uint32_t)cm.W * (uint32_t)cm.H;
    const uint32_t base = (tile - cm.tile_off) * (uint32_t)kPxTile;
    constexpr int NG = kPxPerThread / 4;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const uint32_t idx = base + (uint32_t)g * (kBlock * 4) + threadIdx.x * 4u;
        if (cm.vec_ok && idx + 3 < npx) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            const f4 dv = *glob(reinterpret_cast<const f4*>(cm.depth + idx));
            const f4 cv = *glob(reinterpret_cast<const f4*>(cm.conf + idx));
            t.d[g][0] = dv.x; t.d[g][1] = dv.y; t.d[g][2] = dv.z; t.d[g][3] = dv.w;
            t.c[g][0] = cv.x; t.c[g][1] = cv.y; t.c[g][2] = cv.z; t.c[g][3] = cv.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = idx + j < npx;
                t.d[g][j] = in ? glob(cm.depth)[idx + j] : 0.0f;
                t.c[g][j] = in ? glob(cm.conf)[idx + j] : 0.0f;
            }
        }
    }
}

// the pixels of a loaded tile in order: f(g, j, x, y, depth, confidence, in image, index,
// column ray, row ray), the rays from the camera's ray table `rays` (W column rays, then H
// row rays).  When W and the table's offset are multiples of 4, a thread's 4 pixels share
// a row and their column rays are one 16-byte load.
template <typename F>
__device__ __forceinline__ void visit_tile(const DevCam& cm, uint32_t tile, const TileData& t,
                                           const float* rays, F&& f) {
    const uint32_t npx = (uint32_t)cm.W * (uint32_t)cm.H;
    const uint32_t base = (tile - cm.tile_off) * (uint32_t)kPxTile;
    const uint32_t W = (uint32_t)cm.W;
    const bool quad_rays = ((W | cm.tab_off) & 3u) == 0u;
    constexpr int NG = kPxPerThread / 4;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const uint32_t idx = base + (uint32_t)g * (kBlock * 4) + threadIdx.x * 4u;
        uint32_t y = idx / W;
        uint32_t x = idx - y * W;
        float rxv[4], ryv[4];
        if (quad_rays && idx < npx) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            const f4 r = *glob(reinterpret_cast<const f4*>(rays + x));
            rxv[0] = r.x; rxv[1] = r.y; rxv[2] = r.z; rxv[3] = r.w;
            const float ry = glob(rays)[W + y];
            ryv[0] = ryv[1] = ryv[2] = ryv[3] = ry;
        } else {
            uint32_t xx = x, yy = y;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = idx + j < npx;
                rxv[j] = in ? glob(rays)[xx] : 0.0f;
                ryv[j] = in ? glob(rays)[W + yy] : 0.0f;
                if (++xx == W) { xx = 0; ++yy; }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f(g, j, x, y, t.d[g][j], t.c[g][j], idx + j < npx, idx + j, rxv[j], ryv[j]);
            if (++x == W) { x = 0; ++y; }
        }
    }
}

// every load of the thread first, then the pixels in order: the work on one group does
// not wait for the next group's loads
template <typename F>
__device__ __forceinline__ void for_tile_pixels(const DevCam& cm, uint32_t tile, const float* rays,
                                                F&& f) {
    TileData t;
    load_tile(cm, tile, t);
    visit_tile(cm, tile, t, rays, f);
}

// ---------------------------------------------------------------- Eq. 3 confidence
// Sec. II.2: C = alpha / (1 + beta G) + gamma / (1 + delta sigma_local), divided by
// alpha + gamma so that it lies in (0, 1] as Eq. 2 requires.  G: magnitude of the
// central-difference depth gradient (one-sided where only one neighbour along an axis has
// a valid depth, 0 where none has); sigma_local: population standard deviation of the
// valid depths of the 3x3 window.  Pixels without a valid depth get 0.  float32 with one
// rounding per operation in a fixed order, so the gate and the ranking that use C decide
// exactly as on any other IEEE machine.

__device__ __forceinline__ bool depth_ok(float d) { return __builtin_isfinite(d) && d > 0.0f; }

__device__ __forceinline__ float conf_eq3(const float* D, int W, int H, int x, int y,
                                          const ConfWeights& w) {
    const auto Dg = glob(D);
    const float d = Dg[(size_t)y * (size_t)W + (size_t)x];
    if (!depth_ok(d)) return 0.0f;
    float v[9];
    bool o[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int yy = y + k / 3 - 1, xx = x + k % 3 - 1;
        const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
        const float val = in ? Dg[(size_t)yy * (size_t)W + (size_t)xx] : 0.0f;
        o[k] = in && depth_ok(val);
        v[k] = o[k] ? val : 0.0f;
    }
    // window slots: 1 = (x, y - 1), 3 = (x - 1, y), 5 = (x + 1, y), 7 = (x, y + 1)
    const float gx = (o[5] && o[3]) ? (v[5] - v[3]) * 0.5f
                                    : (o[5] ? v[5] - d : (o[3] ? d - v[3] : 0.0f));
    const float gy = (o[7] && o[1]) ? (v[7] - v[1]) * 0.5f
                                    : (o[7] ? v[7] - d : (o[1] ? d - v[1] : 0.0f));
    const float G = sqrtf(gx * gx + gy * gy);
    float n = 0.0f, s = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (o[k]) {
            n = n + 1.0f;
            s = s + v[k];
        }
    }
    const float mean = s / n;
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (o[k]) {
            const float e = v[k] - mean;
            acc = acc + e * e;
        }
    }
    const float sd = sqrtf(acc / n);
    const float t1 = w.a / (1.0f + w.b * G);
    const float t2 = w.g / (1.0f + w.d * sd);
    return (t1 + t2) / (w.a + w.g);
}

// per 4096-pixel tile (the same pixel walk as the other per-pixel phases): C into the
// camera's conf_out, with the paper's weights
__device__ __forceinline__ void ph_conf(const Ctx& C, uint32_t tile, char*) {
    const DevCam& cm = C.cams[cam_of_tile(C, tile)];
    if (!cm.conf_out) return;
    const ConfWeights w{0.5f, 0.5f, 1.0f, 1.0f};
    const uint32_t npx = (uint32_t)cm.W * (uint32_t)cm.H;
    const uint32_t base = (tile - cm.tile_off) * (uint32_t)kPxTile;
    const uint32_t W = (uint32_t)cm.W;
    for (int g = 0; g < kPxPerThread / 4; ++g) {
        const uint32_t idx0 = base + (uint32_t)g * (kBlock * 4) + threadIdx.x * 4u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t idx = idx0 + j;
            if (idx >= npx) break;
            const uint32_t y = idx / W, x = idx - y * W;
            glob(cm.conf_out)[idx] = conf_eq3(cm.depth, cm.W, cm.H, (int)x, (int)y, w);
        }
    }
}

// ---------------------------------------------------------------- Eq. 12 evaluator
// Multi-camera depth consistency of one fused point: over the cameras that see it (in
// front, nearest pixel inside the image, valid depth there, not occluded: z <= D + c z^2)
// the sum of |z - D| (double) and their number.  Projection as in Eq. 4 (float32, one
// rounding per operation, the same order as the per-cell phase).
__device__ __forceinline__ void emc_point(const DevCam* cams, int ncams, const Pt& p, float c_occ,
                                          double& err, uint32_t& cnt) {
    err = 0.0;
    cnt = 0;
    for (int i = 0; i < ncams; ++i) {
        const DevCam& cm = cams[i];
        const float Z = ((cm.R[6] * p.x + cm.R[7] * p.y) + cm.R[8] * p.z) + cm.t[2];
        if (!(Z > 0.0f)) continue;
        const float X = ((cm.R[0] * p.x + cm.R[1] * p.y) + cm.R[2] * p.z) + cm.t[0];
        const float Y = ((cm.R[3] * p.x + cm.R[4] * p.y) + cm.R[5] * p.z) + cm.t[1];
        const float u = cm.fx * (X / Z) + cm.cx, v = cm.fy * (Y / Z) + cm.cy;
        const float fu = floorf(u + 0.5f), fv = floorf(v + 0.5f);
        if (!(fu >= 0.0f && fu < (float)cm.W && fv >= 0.0f && fv < (float)cm.H)) continue;
        const float d = glob(cm.depth)[(size_t)fv * (size_t)cm.W + (size_t)fu];
        if (!depth_ok(d)) continue;
        const float tol = (c_occ * Z) * Z;
        if (!(Z <= d + tol)) continue;
        err += fabs((double)Z - (double)d);
        ++cnt;
    }
}

// ---------------------------------------------------------------- phase: camera prep
// One workgroup per camera: the centre c = -R^T t (Eq. 8's inverse extrinsics), the rank
// of the camera in its frame under (centre x, y, z, index) used to break distance ties,
// the staged copy used by the per-cell phase, and the ray tables (x - cx)/fx per column
// and (y - cy)/fy per row, so that no per-pixel step divides.

__device__ __forceinline__ void ph_cam_prep(const Ctx& C, uint32_t i, char* smem) {
    if (i == 0 && threadIdx.x == 0) {
        // the call's batch-wide state, read or counted by every later launch of the call
        BatchState& bs = *C.bs;
        bs.M_tot = 0; bs.S_tot = 0; bs.error = 0; bs.key64 = 0;
        bs.key_bits = 0; bs.npass = 0; bs.T_tot = 0;
    }
    DevCam& cm = C.cams[i];
    const DevFrame& fr = C.frames[cm.frame];
    uint32_t* s_w = reinterpret_cast<uint32_t*>(smem);
    DevCam me = cm;
    camera_centre(me);
    // rank: count the frame's cameras that come first
    uint32_t before = 0;
    for (uint32_t j = fr.cam_begin + threadIdx.x; j < fr.cam_begin + fr.n_cams; j += kBlock) {
        DevCam o = C.cams[j];
        camera_centre(o);
        bool b;
        if (o.c[0] != me.c[0]) b = o.c[0] < me.c[0];
        else if (o.c[1] != me.c[1]) b = o.c[1] < me.c[1];
        else if (o.c[2] != me.c[2]) b = o.c[2] < me.c[2];
        else b = j < i;
        before += b ? 1u : 0u;
    }
    const uint32_t rank = block_sum(before, s_w);
    float* rx = C.raytab + cm.tab_off;
    float* ry = rx + cm.W;
    for (int x = threadIdx.x; x < cm.W; x += kBlock) rx[x] = ((float)x - me.cx) / me.fx;
    for (int y = threadIdx.x; y < cm.H; y += kBlock) ry[y] = ((float)y - me.cy) / me.fy;
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) cm.c[a] = me.c[a];
        cm.rank = rank;
        CamLite cl;
        for (int a = 0; a < 9; ++a) cl.R[a] = me.R[a];
        for (int a = 0; a < 3; ++a) { cl.t[a] = me.t[a]; cl.c[a] = me.c[a]; }
        cl.fx = me.fx; cl.fy = me.fy; cl.cx = me.cx; cl.cy = me.cy;
        cl.W = me.W; cl.H = me.H; cl.rank = rank; cl.pix_off = me.pix_off;
        cl.frame = me.frame;
        cl.frame_cam = i - fr.cam_begin;
        cl.tab_off = cm.tab_off;
        cl.invW = 1.0f / (float)me.W;
        cl.cxh = me.cx + 0.5f;
        cl.cyh = me.cy + 0.5f;
        const float Wf = (float)me.W, Hf = (float)me.H;      // exact: sides <= 2^14
        cl.in_hx = float_below(Wf - kFovMargin);
        cl.in_hy = float_below(Hf - kFovMargin);
        cl.out_hx = float_below(Wf + kFovMargin);
        cl.out_hy = float_below(Hf + kFovMargin);
        cl.depth = me.depth; cl.conf = me.conf; cl.rgb = me.rgb;
        C.camlite[i] = cl;
    }
}

// ---------------------------------------------------------------- phase: back-project + AABB
// Eq. 8-9 per pixel, and the extents of Sec. II.5(1)b as per-tile partials (no atomics).
// Also clears this tile's share of the coarse histogram's copies for the next phases.

__device__ __forceinline__ void ph_backproject(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    const uint32_t tid = threadIdx.x;
    if (!(P.flags & 4u)) {
        const uint64_t nc = (uint64_t)H.n_counts * kCountStripes;
        const uint64_t chunk = (nc + H.n_px_tiles - 1) / H.n_px_tiles;
        const uint64_t b0 = (uint64_t)tile * chunk, b1 = min(nc, b0 + chunk);
        for (uint64_t i = b0 + tid; i < b1; i += kBlock) C.counts[i] = 0;
    }
    const DevCam& cm = C.cams[cam_of_tile(C, tile)];
    const float* rx = C.raytab + cm.tab_off;          // the camera's ray table
    const bool no_mf = P.flags & 1u;
    uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u}, cnt = 0;
    for_tile_pixels(cm, tile, rx, [&](int, int, uint32_t, uint32_t, float d, float c, bool in,
                                      uint32_t, float rxj, float ryj) {
        if (!in || !gate_px(d, c, P.tau, no_mf)) return;
        const Pt p = backproject_ray(cm, rxj, ryj, d);
        if (!finite3(p)) return;
        const uint32_t o[3] = {f2o(p.x), f2o(p.y), f2o(p.z)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = o[a] < mn[a] ? o[a] : mn[a];
            mx[a] = o[a] > mx[a] ? o[a] : mx[a];
        }
        ++cnt;
    });
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
    uint32_t* s = reinterpret_cast<uint32_t*>(smem);     // [4][8]
    const uint32_t w = tid / kWave;
    if (lane_id() == 0) {
        for (int a = 0; a < 3; ++a) { s[w * 8 + a] = mn[a]; s[w * 8 + 3 + a] = mx[a]; }
        s[w * 8 + 6] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        TilePart tp;
        for (int a = 0; a < 3; ++a) {
            tp.mn[a] = min(min(s[a], s[8 + a]), min(s[16 + a], s[24 + a]));
            tp.mx[a] = max(max(s[3 + a], s[11 + a]), max(s[19 + a], s[27 + a]));
        }
        tp.cnt = s[6] + s[14] + s[22] + s[30];
        tp.pad = 0;
        C.tiles[tile] = tp;
    }
}

// ---------------------------------------------------------------- phase: per-frame reduce
// One workgroup per frame: the frame's AABB, point count and coarse grid (Sec. II.5(1)b-c)
// and the frame-local compaction offset of every pixel tile.  The frames' first compacted
// positions (prefix of the counts over frames) are added by the keys phase.

__device__ __forceinline__ void ph_tile_reduce(const Ctx& C, uint32_t f, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    if (f >= H.n_frames) return;
    const uint32_t tid = threadIdx.x, w = tid / kWave;
    uint32_t* s_w = reinterpret_cast<uint32_t*>(smem);          // [8]
    uint32_t* s_r = s_w + 8;                                    // [4][8]
    const DevFrame& fr = C.frames[f];
    uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u};
    uint32_t carry = 0;
    // 8 consecutive tiles per thread per step: their loads are in flight together
    constexpr int kPer = 8;
    for (uint32_t b = 0; b < fr.n_tiles; b += kBlock * kPer) {
        uint32_t c[kPer], sum = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t i = b + tid * kPer + j;
            const bool in = i < fr.n_tiles;
            TilePart tp;
            if (in) tp = C.tiles[fr.tile_begin + i];
            c[j] = in ? tp.cnt : 0u;
            if (in && c[j]) {
                for (int a = 0; a < 3; ++a) {
                    mn[a] = min(mn[a], tp.mn[a]);
                    mx[a] = max(mx[a], tp.mx[a]);
                }
            }
            sum += c[j];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl(sum, s_w, tot);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t i = b + tid * kPer + j;
            if (i < fr.n_tiles) C.tile_off[fr.tile_begin + i] = run;
            run += c[j];
        }
        carry += tot;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = min(mn[a], (uint32_t)__shfl_xor(mn[a], o));
            mx[a] = max(mx[a], (uint32_t)__shfl_xor(mx[a], o));
        }
    }
    if (lane_id() == 0)
        for (int a = 0; a < 3; ++a) { s_r[w * 8 + a] = mn[a]; s_r[w * 8 + 3 + a] = mx[a]; }
    __syncthreads();
    if (tid == 0) {
        FrameState& st = C.fs[f];
        float lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            st.bmin_o[a] = min(min(s_r[a], s_r[8 + a]), min(s_r[16 + a], s_r[24 + a]));
            st.bmax_o[a] = max(max(s_r[3 + a], s_r[11 + a]), max(s_r[19 + a], s_r[27 + a]));
            lo[a] = o2f(st.bmin_o[a]);
            hi[a] = o2f(st.bmax_o[a]);
            st.bmin[a] = lo[a];
        }
        st.e = coarse_exponent(lo, hi, P.log2G);
        st.scale = __uint_as_float((uint32_t)(127 - st.e) << 23);
        st.M = carry;
        st.cell_begin = 0;
        st.has_cells = 0;
        st.fine_begin = 0;
        for (int k = 0; k < kRSlots; ++k) st.R[k] = 0;
    }
}

// ---------------------------------------------------------------- phase: coarse histogram
// Sec. II.5(1)c.  Counts are merged per thread (4 neighbouring pixels), then per run of
// lanes with the same cell (a wave scan), accumulated in an LDS hash of the tile's cells,
// and one global atomic per distinct cell and tile goes out at the end.  A frame occupies
// only a few thousand coarse cells, so those atomics meet on few addresses, and device-
// scope atomics on one address serialise: workgroup w adds into copy w mod kCountStripes
// of the counts, and the first scan phase folds the copies into copy 0.

// one pixel tile into the LDS hash (counts: the frame's, for the rare full-hash case)
__device__ __forceinline__ void hist_tile(const Ctx& C, const DevCam& cm, uint32_t tile,
                                          const TileData& td, uint32_t* s_key, uint32_t* s_cnt,
                                          uint32_t* counts, bool no_mf) {
    const DevParams& P = C.hdr->prm;
    const float* rx = C.raytab + cm.tab_off;          // the camera's ray table
    FrameGrid g;
    frame_grid(C.fs[cm.frame], P, g);
    // add n points of cell `key` to the tile's LDS hash (global atomic if the hash is full)
    auto hash_add = [&](uint32_t key, uint32_t n) {
        uint32_t h = (key * 2654435761u) >> (32 - 11);
        for (int probe = 0; probe < 32; ++probe) {
            const uint32_t old = atomicCAS(&s_key[h], kPad, key);
            if (old == kPad || old == key) {
                atomicAdd(&s_cnt[h], n);
                return;
            }
            h = (h + 1) & (kHashSlots - 1);
        }
        atomicAdd(&counts[key], n);
    };
    // consecutive lanes hold consecutive pixels, so equal cells come in runs of lanes: a
    // wave scan sums each run and only its last lane touches the hash (every lane calls)
    auto run_add = [&](uint32_t key, uint32_t n) {
        const uint32_t l = lane_id();
        const uint32_t kk = n ? key : kPad;            // lanes without points end runs
        const uint32_t prev = __shfl_up(kk, 1), next = __shfl_down(kk, 1);
        const bool head = l == 0 || prev != kk;
        const bool tail = l == 63 || next != kk;
        const uint32_t incl = wave_incl(n);
        // first lane of this lane's run: the highest run head at or below it (lane 0 is one)
        const uint64_t heads = __ballot(head);
        const uint64_t le = l == 63u ? ~0ull : ((2ull << l) - 1ull);
        const uint32_t hs = 63u - (uint32_t)__clzll((long long)(heads & le));
        const uint32_t before = __shfl(incl, hs == 0 ? 0 : (int)hs - 1);
        const uint32_t tot = incl - (hs == 0 ? 0u : before);
        if (tail && kk != kPad && tot) hash_add(key, tot);
    };
    uint32_t kk[4];
    bool hv[4];
    visit_tile(cm, tile, td, rx, [&](int, int j, uint32_t, uint32_t, float d, float c, bool in,
                                     uint32_t, float rxj, float ryj) {
        bool has = in && gate_px(d, c, P.tau, no_mf);
        uint32_t key = 0;
        if (has) {
            const Pt p = backproject_ray(cm, rxj, ryj, d);
            has = finite3(p);
            if (has) key = coarse_cell(g, p).lin;
        }
        kk[j] = key;
        hv[j] = has;
        if (j == 3) {
            // a thread's 4 neighbouring pixels nearly always share their coarse cell:
            // merge them first, then the rare others one by one
            uint32_t k0 = 0, n0 = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (hv[q] && (n0 == 0 || kk[q] == k0)) {
                    k0 = kk[q];
                    ++n0;
                    hv[q] = false;
                }
            }
            run_add(k0, n0);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (hv[q]) hash_add(kk[q], 1u);
        }
    });
}

__device__ __forceinline__ void ph_hist(const Ctx& C, uint32_t item, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    if (P.flags & 4u) return;
    uint32_t* s_key = reinterpret_cast<uint32_t*>(smem);
    uint32_t* s_cnt = s_key + kHashSlots;
    for (uint32_t i = threadIdx.x; i < kHashSlots; i += kBlock) {
        s_key[i] = kPad;
        s_cnt[i] = 0;
    }
    __syncthreads();
    const bool no_mf = P.flags & 1u;
    const uint64_t G3 = (uint64_t)(P.G * P.G * P.G);
    // this workgroup's tiles share one LDS hash; it goes out to the frame's counts (one
    // global atomic per distinct cell) when the frame changes and at the end
    const uint32_t t0 = item * H.hist_tiles;
    const uint32_t t1 = min(t0 + H.hist_tiles, H.n_px_tiles);
    if (t0 >= t1) return;
    uint32_t frame = C.cams[cam_of_tile(C, t0)].frame;
    uint32_t* const stripe = C.counts + (uint64_t)(item % kCountStripes) * H.n_counts;
    auto flush = [&](uint32_t f) {
        __syncthreads();
        uint32_t* counts = stripe + (uint64_t)f * G3;
        for (uint32_t i = threadIdx.x; i < kHashSlots; i += kBlock) {
            const uint32_t k = s_key[i];
            if (k != kPad) atomicAdd(&counts[k], s_cnt[i]);
            s_key[i] = kPad;
            s_cnt[i] = 0;
        }
        __syncthreads();
    };
    // the next tile's loads are issued before this tile's work (two buffers in registers)
    TileData buf[2];
    const DevCam* cur = &C.cams[cam_of_tile(C, t0)];
    load_tile(*cur, t0, buf[0]);
#pragma unroll
    for (int i = 0; i < kMaxHistTiles; ++i) {
        const uint32_t tile = t0 + (uint32_t)i;
        if (tile >= t1) break;
        const DevCam& cm = *cur;
        if (tile + 1 < t1) {
            cur = &C.cams[cam_of_tile(C, tile + 1)];
            load_tile(*cur, tile + 1, buf[(i + 1) & 1]);
        }
        if (cm.frame != frame) {
            flush(frame);
            frame = cm.frame;
        }
        hist_tile(C, cm, tile, buf[i & 1], s_key, s_cnt, stripe + (uint64_t)cm.frame * G3,
                  no_mf);
    }
    flush(frame);
}

// ---------------------------------------------------------------- field-of-view classes
// For an occupied coarse cell and each camera of its frame: is every point of the cell in
// view by the exact float32 test of Eq. 4 (in front, nearest pixel floor(u + 1/2) inside
// the image), is none, or neither?  The points of coarse cell ci satisfy
// floor((p - bmin) 2^-e) = ci with one rounding in the subtraction, so they lie in the box
// bmin + [ci, ci + 1] s0 widened by that rounding.  Over a box entirely in front of the
// camera, the projection is a projective map, which takes the box's convex hull to the
// convex hull of its corners' images: u and v over the box lie between their values at
// the eight corners.  Those are computed in double, and a decision is taken only with a
// margin far above the float32 error of the per-point computation (a few units in the
// last place of the terms of X, Y, Z, the quotient and the sums), so a class never
// disagrees with the exact per-point test; everything else is "partial" and takes that
// test.
__device__ __forceinline__ void classify_box(const DevCam& cm, const double lo[3],
                                             const double hi[3], bool& in_all, bool& partial) {
    in_all = false;
    partial = false;
    double zmin = INFINITY, zmax = -INFINITY, umin = INFINITY, umax = -INFINITY;
    double vmin = INFINITY, vmax = -INFINITY, mx = 0.0, mz = 0.0;
    for (int k = 0; k < 8; ++k) {
        const double q0 = (k & 1) ? hi[0] : lo[0];
        const double q1 = (k & 2) ? hi[1] : lo[1];
        const double q2 = (k & 4) ? hi[2] : lo[2];
        const double r0 = (double)cm.R[0] * q0, r1 = (double)cm.R[1] * q1, r2 = (double)cm.R[2] * q2;
        const double r3 = (double)cm.R[3] * q0, r4 = (double)cm.R[4] * q1, r5 = (double)cm.R[5] * q2;
        const double r6 = (double)cm.R[6] * q0, r7 = (double)cm.R[7] * q1, r8 = (double)cm.R[8] * q2;
        const double X = ((r0 + r1) + r2) + (double)cm.t[0];
        const double Y = ((r3 + r4) + r5) + (double)cm.t[1];
        const double Z = ((r6 + r7) + r8) + (double)cm.t[2];
        // magnitudes of the terms of X, Y, Z (their float32 rounding is relative to these)
        const double ax = fabs(r0) + fabs(r1) + fabs(r2) + fabs((double)cm.t[0]);
        const double ay = fabs(r3) + fabs(r4) + fabs(r5) + fabs((double)cm.t[1]);
        const double az = fabs(r6) + fabs(r7) + fabs(r8) + fabs((double)cm.t[2]);
        mx = fmax(mx, fmax(ax, ay));
        mz = fmax(mz, az);
        zmin = fmin(zmin, Z);
        zmax = fmax(zmax, Z);
        if (Z > 0.0) {
            const double rz = 1.0 / Z;
            const double u = (double)cm.fx * (X * rz) + (double)cm.cx;
            const double v = (double)cm.fy * (Y * rz) + (double)cm.cy;
            umin = fmin(umin, u); umax = fmax(umax, u);
            vmin = fmin(vmin, v); vmax = fmax(vmax, v);
        }
    }
    // Far from the float32 range limits the per-point error is relative to the terms;
    // near them (overflow of a term, subnormal terms) no class is claimed.
    if (!(mx <= 1e36 && mz <= 1e36)) { partial = true; return; }
    const double ez = 1e-5 * mz + 1e-30;               // >> float32 error of Z
    if (zmax < -ez) return;                            // wholly behind: sees none
    if (!(zmin > ez)) { partial = true; return; }      // straddles Z = 0
    // The float32 u of a point differs from the real one by at most about
    // 4e-7 (|f| mx + |u - c| mz) / Z (errors of X and Z carried through X / Z and the
    // scaling by f) plus a few roundings of |u|: margins 25 times that, plus 1/16 px.
    const double eu = fmax(fabs(umin - (double)cm.cx), fabs(umax - (double)cm.cx));
    const double ev = fmax(fabs(vmin - (double)cm.cy), fabs(vmax - (double)cm.cy));
    const double du = 1e-5 * ((fabs((double)cm.fx) * mx + eu * mz) / zmin + fabs(umin) +
                              fabs(umax) + fabs((double)cm.cx)) + 0.0625;
    const double dv = 1e-5 * ((fabs((double)cm.fy) * mx + ev * mz) / zmin + fabs(vmin) +
                              fabs(vmax) + fabs((double)cm.cy)) + 0.0625;
    const double W = (double)cm.W, H = (double)cm.H;
    const bool in = umin >= -0.5 + du && umax <= W - 0.5 - du && vmin >= -0.5 + dv &&
                    vmax <= H - 0.5 - dv;
    const bool out = umax < -0.5 - du || umin > W - 0.5 + du || vmax < -0.5 - dv ||
                     vmin > H - 0.5 + dv;
    in_all = in;
    partial = !in && !out;
}

// ---------------------------------------------------------------- phase: coarse scan
// span(c) = 8^L(c) dense fine indices for every occupied coarse cell; the exclusive scan
// over (frame, cell) gives each cell's first dense index.  Three steps: tile sums (which
// also fold the histogram's copies of the counts), a one-workgroup scan of the tile sums
// (which also fixes the sort's key width and passes), and the per-tile scan.

__device__ __forceinline__ uint64_t span_of(uint32_t n, const DevParams& P) {
    return n ? (1ull << (3 * level_of(n, P))) : 0ull;
}

__device__ __forceinline__ void ph_scan_a(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    const uint64_t total = H.n_counts;
    uint64_t s = 0;
    const uint64_t base = (uint64_t)tile * kScanTile;
#pragma unroll 4
    for (int i = 0; i < kScanTile / kBlock; ++i) {
        const uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
        if (idx < total) {
            uint32_t n = 0;                    // fold the histogram's copies into copy 0
#pragma unroll
            for (int q = 0; q < kCountStripes; ++q) n += C.counts[idx + (uint64_t)q * total];
            C.counts[idx] = n;
            s += span_of(n, P);
        }
    }
    uint64_t* s_w = reinterpret_cast<uint64_t*>(smem);
    s = wave_sum64(s);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) C.scan_tile[tile] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__device__ __forceinline__ void ph_scan_m(const Ctx& C, uint32_t, char* smem) {
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
        uint32_t bits = carry > 1 ? 64u - (uint32_t)__clzll((long long)(carry - 1)) : 0u;
        if (bits > 32u && !H.key64_ok) {   // cannot happen: the bound fixed 32-bit keys (and
            raise_error(C.bs, kErrBounds); // the scatter's staging size); stay within it
            bits = 32u;
        }
        bs.key_bits = bits;
        bs.key64 = bits > 32 ? 1u : 0u;
        const uint32_t mb = H.max_radix_bits;
        uint32_t np = (bits + mb - 1) / mb;
        if (np > H.npass_max) {           // cannot happen: npass_max bounds the key width
            raise_error(C.bs, kErrBounds);
            np = H.npass_max;
        }
        bs.npass = np;
        // spread the key bits evenly over the passes (fewest passes, narrowest digits)
        uint32_t shift = 0;
        for (uint32_t k = 0; k < np; ++k) {
            const uint32_t w = bits / np + (k < bits % np ? 1u : 0u);
            bs.pass_shift[k] = shift;
            bs.pass_bits[k] = w;
            shift += w;
        }
    }
}

__device__ __forceinline__ void ph_scan_b(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    const uint64_t per_frame = (uint64_t)(P.G * P.G * P.G);
    const uint64_t total = H.n_counts;
    uint64_t* s_w = reinterpret_cast<uint64_t*>(smem);
    constexpr int kPer = kScanTile / kBlock;       // consecutive cells per thread
    const uint64_t base = (uint64_t)tile * kScanTile + (uint64_t)threadIdx.x * kPer;
    uint64_t sp[kPer];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const uint64_t idx = base + i;
        const uint32_t n = idx < total ? C.counts[idx] : 0u;
        const int L = n ? level_of(n, P) : 0;
        sp[i] = n ? (1ull << (3 * L)) : 0ull;
        if (idx < total) C.level[idx] = (uint8_t)L;
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

// One thread per (coarse cell, camera slot): the field-of-view class of each camera of the
// frame for every occupied coarse cell (the per-cell phase reads the class of each
// representative's coarse cell).  The camera slots of a cell are consecutive lanes of one
// wave (2^cls_lanes of them, at least the frame's camera count), so two ballots assemble
// the cell's masks.
__device__ __forceinline__ void ph_class(const Ctx& C, uint32_t item, char*) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    if (P.flags & 6u) return;                 // no V (NO_DC) or no grid (NO_SA)
    const uint32_t lanes = H.cls_lanes;
    const uint64_t t = (uint64_t)item * kBlock + threadIdx.x;
    const uint64_t idx = t >> lanes;
    const uint32_t jj = (uint32_t)(t & ((1u << lanes) - 1u));
    const uint64_t per_frame = (uint64_t)(P.G * P.G * P.G);
    bool occ = idx < (uint64_t)H.n_counts && C.counts[idx] != 0u;
    bool in = false, part = false;
    if (occ) {
        const uint32_t f = (uint32_t)(idx / per_frame);
        const uint32_t lin = (uint32_t)(idx - (uint64_t)f * per_frame);
        const DevFrame& fr = C.frames[f];
        if (jj < fr.n_cams) {
            const FrameState& st = C.fs[f];
            const uint32_t G = (uint32_t)P.G;
            const uint32_t ci[3] = {lin % G, (lin / G) % G, lin / (G * G)};
            const double s0 = 1.0 / (double)st.scale;          // 2^e, exact
            double lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                const double b = (double)st.bmin[a], bx = (double)o2f(st.bmax_o[a]);
                // widened by the rounding of p - bmin (at most 2^-24 of |p - bmin|)
                const double eps = 0x1p-22 * (fabs(bx - b) + (double)G * s0) + 0x1p-22 * fabs(b);
                lo[a] = b + (double)ci[a] * s0 - eps;
                hi[a] = b + (double)(ci[a] + 1) * s0 + eps;
                // the last cell also holds every point beyond the grid (a clamped exponent
                // leaves the extent wider than G s0): up to the frame's maximum
                if (ci[a] == G - 1) hi[a] = fmax(hi[a], bx + eps);
            }
            classify_box(C.cams[fr.cam_begin + jj], lo, hi, in, part);
        }
    }
    const uint64_t bin = __ballot(in), bpart = __ballot(part);
    const uint32_t l = lane_id(), base = l & ~((1u << lanes) - 1u);
    if (occ && jj == 0) {
        const uint64_t m = lanes >= 6 ? ~0ull : ((1ull << (1u << lanes)) - 1ull);
        CamClass cc;
        cc.in_all = (bin >> base) & m;
        cc.partial = (bpart >> base) & m;
        C.cls[idx] = cc;
    }
}

// ---------------------------------------------------------------- phase: keys
// Sec. II.5(1)e: every gated point gets its cell's dense index (order-preserving image of the
// canonical key); points are compacted in pixel order at the tile's precomputed offset.

__device__ __forceinline__ void ph_keys(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    BatchState* bs = C.bs;
    const DevCam& cm = C.cams[cam_of_tile(C, tile)];
    const bool no_mf = P.flags & 1u;
    const bool no_sa = P.flags & 4u;
    const uint32_t G3 = (uint32_t)(P.G * P.G * P.G);
    const uint8_t* lvl = C.level + (uint64_t)cm.frame * G3;
    const uint64_t* fbase = C.fine_base + (uint64_t)cm.frame * G3;
    const bool key64 = bs->key64;
    uint32_t* s_w = reinterpret_cast<uint32_t*>(smem);
    const float* rx = C.raytab + cm.tab_off;          // the camera's ray table
    FrameGrid g;
    if (!no_sa) frame_grid(C.fs[cm.frame], P, g);

    if (tile == 0) {
        // every frame's first compacted position and the batch's point count, for the phases
        // after this one
        for (uint32_t f = threadIdx.x; f < H.n_frames; f += kBlock) {
            uint32_t k = 0;
            for (uint32_t h = 0; h < f; ++h) k += C.fs[h].M;
            C.fs[f].key_begin = k;
        }
        if (threadIdx.x == 0) {
            uint32_t m = 0;
            for (uint32_t h = 0; h < H.n_frames; ++h) m += C.fs[h].M;
            bs->M_tot = m;
        }
    }

    uint64_t kv[kPxPerThread];
    uint32_t mask = 0;
    for_tile_pixels(cm, tile, rx, [&](int gi, int j, uint32_t, uint32_t, float d, float c,
                                      bool in, uint32_t, float rxj, float ryj) {
        const int k = gi * 4 + j;
        kv[k] = 0;
        if (!in || !gate_px(d, c, P.tau, no_mf)) return;
        const Pt p = backproject_ray(cm, rxj, ryj, d);
        if (!finite3(p)) return;
        mask |= 1u << k;
        if (no_sa) return;
        const CellCoord cc = coarse_cell(g, p);
        const int L = lvl[cc.lin];
        int loc[3];
        fine_local(cc, L, loc);
        kv[k] = fbase[cc.lin] +
                ((((uint64_t)loc[2] << L) | (uint64_t)loc[1]) << L | (uint64_t)loc[0]);
    });
    // ranks in pixel order: group-major, then thread, then j.  One scan of the four group
    // counts packed in 16-bit fields (a group holds at most 1024 points per tile)
    uint64_t packed = 0;
#pragma unroll
    for (int gi = 0; gi < 4; ++gi)
        packed |= (uint64_t)__popc((mask >> (gi * 4)) & 0xFu) << (16 * gi);
    uint64_t ptot;
    const uint64_t pex = block_excl64(packed, reinterpret_cast<uint64_t*>(s_w), ptot);
    uint32_t off[4], tile_total = 0;
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
        off[gi] = tile_total + (uint32_t)((pex >> (16 * gi)) & 0xFFFFu);
        tile_total += (uint32_t)((ptot >> (16 * gi)) & 0xFFFFu);
    }
    // the frame's first compacted position: the points of the frames before it (each wave
    // sums them itself; at most kMaxFrames counts)
    uint32_t kb = 0;
    for (uint32_t g = lane_id(); g < cm.frame; g += kWave) kb += C.fs[g].M;
    kb = (uint32_t)wave_sum64(kb);
    const uint32_t pre = kb + C.tile_off[tile];
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
            ++o;
        }
    }
}

// ---------------------------------------------------------------- LSD radix sort
// Reduce-then-scan per pass: tile digit histograms (UP), a scan of each digit's row over
// the tiles (SCAN), and a stable scatter (DOWN) that ranks keys inside the tile by
// wave-level digit matching and stages them in LDS so writes leave in digit runs.

__device__ __forceinline__ uint32_t n_keys(const Ctx& C) { return min(C.bs->M_tot, C.P_cap); }

template <int ITEMS>
__device__ __forceinline__ uint32_t n_sort_tiles_real(const Ctx& C) {
    return (n_keys(C) + kBlock * ITEMS - 1) / (kBlock * ITEMS);
}

__device__ __forceinline__ uint64_t load_key(const Ctx& C, bool from_b, bool key64, uint32_t i) {
    const void* k = from_b ? C.keysB : C.keysA;
    return key64 ? reinterpret_cast<const uint64_t*>(k)[i]
                 : (uint64_t)reinterpret_cast<const uint32_t*>(k)[i];
}

// In-place exclusive scan of an LDS array of D <= kMaxDigits entries; returns the total.
__device__ __forceinline__ uint32_t lds_excl_scan(uint32_t* a, uint32_t D, uint32_t* s_w) {
    const uint32_t per = (D + kBlock - 1) / kBlock;
    const uint32_t b = threadIdx.x * per;
    uint32_t loc = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (b + j < D) loc += a[b + j];
    uint32_t tot;
    uint32_t run = block_excl(loc, s_w, tot);
    for (uint32_t j = 0; j < per; ++j) {
        if (b + j < D) {
            const uint32_t v = a[b + j];
            a[b + j] = run;
            run += v;
        }
    }
    __syncthreads();
    return tot;
}

template <int ITEMS>
__device__ __forceinline__ void ph_radix_up(const Ctx& C, uint32_t pass, uint32_t tile, char* smem) {
    constexpr int KT = kBlock * ITEMS;
    BatchState* bs = C.bs;
    if ((C.hdr->prm.flags & 4u) || pass >= bs->npass) return;
    const uint32_t n = n_keys(C), nt = n_sort_tiles_real<ITEMS>(C);
    if (tile >= nt) return;
    const uint32_t bits = bs->pass_bits[pass], shift = bs->pass_shift[pass], D = 1u << bits;
    const bool key64 = bs->key64, from_b = pass & 1;
    uint32_t* s_h = reinterpret_cast<uint32_t*>(smem);
    for (uint32_t d = threadIdx.x; d < D; d += kBlock) s_h[d] = 0;
    __syncthreads();
    if (!key64) {
        // a histogram does not care about order: each thread counts ITEMS consecutive keys,
        // read as 16-byte vectors (2 KiB per wave load instead of 256 bytes)
        const uint32_t* kp = reinterpret_cast<const uint32_t*>(from_b ? C.keysB : C.keysA);
        const uint32_t b = tile * KT + threadIdx.x * ITEMS;
        if (b + ITEMS <= n) {
            typedef uint32_t u4 __attribute__((ext_vector_type(4)));
            u4 v[ITEMS / 4];
#pragma unroll
            for (int q = 0; q < ITEMS / 4; ++q) v[q] = glob(reinterpret_cast<const u4*>(kp + b))[q];
#pragma unroll
            for (int q = 0; q < ITEMS / 4; ++q) {
                atomicAdd(&s_h[(v[q].x >> shift) & (D - 1)], 1u);
                atomicAdd(&s_h[(v[q].y >> shift) & (D - 1)], 1u);
                atomicAdd(&s_h[(v[q].z >> shift) & (D - 1)], 1u);
                atomicAdd(&s_h[(v[q].w >> shift) & (D - 1)], 1u);
            }
        } else {
            for (int i = 0; i < ITEMS; ++i)
                if (b + (uint32_t)i < n) atomicAdd(&s_h[(glob(kp)[b + i] >> shift) & (D - 1)], 1u);
        }
    } else {
#pragma unroll 4
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = tile * KT + (uint32_t)i * kBlock + threadIdx.x;
            if (idx < n) atomicAdd(&s_h[(uint32_t)(load_key(C, from_b, true, idx) >> shift) & (D - 1)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < D; d += kBlock) C.digit_hist[(uint64_t)d * nt + tile] = s_h[d];
}

// In-place exclusive scan of row[0, n) by one workgroup, for n <= kBlock * kRowScanPer:
// thread t takes the ceil(n / kBlock) consecutive entries from t ceil(n / kBlock), and all
// of its loads are in flight before the one block scan.  Returns the total.
constexpr int kRowScanPer = 32;
__device__ __forceinline__ uint32_t row_scan_one_step(uint32_t* row, uint32_t n, uint32_t* s_w) {
    const uint32_t per = (n + kBlock - 1) / kBlock;
    const uint32_t b = threadIdx.x * per;
    uint32_t v[kRowScanPer], loc = 0;
#pragma unroll
    for (int j = 0; j < kRowScanPer; ++j) {
        const uint32_t i = b + (uint32_t)j;
        v[j] = ((uint32_t)j < per && i < n) ? row[i] : 0u;
        loc += v[j];
    }
    uint32_t tot;
    uint32_t run = block_excl(loc, s_w, tot);
#pragma unroll
    for (int j = 0; j < kRowScanPer; ++j) {
        const uint32_t i = b + (uint32_t)j;
        if ((uint32_t)j < per && i < n) row[i] = run;
        run += v[j];
    }
    return tot;
}

template <int ITEMS>
__device__ __forceinline__ void ph_radix_scan(const Ctx& C, uint32_t pass, uint32_t d, char* smem) {
    BatchState* bs = C.bs;
    if ((C.hdr->prm.flags & 4u) || pass >= bs->npass) return;
    const uint32_t D = 1u << bs->pass_bits[pass];
    if (d >= D) return;
    const uint32_t nt = n_sort_tiles_real<ITEMS>(C);
    uint32_t* row = C.digit_hist + (uint64_t)d * nt;
    uint32_t* s_w = reinterpret_cast<uint32_t*>(smem);
    if (nt <= (uint32_t)(kBlock * kRowScanPer)) {
        const uint32_t tot = row_scan_one_step(row, nt, s_w);
        if (threadIdx.x == 0) C.digit_total[d] = tot;
        return;
    }
    uint32_t carry = 0;
    constexpr int kPer = 8;                  // consecutive tiles per thread per step
    for (uint32_t b = 0; b < nt; b += kBlock * kPer) {
        uint32_t v[kPer], loc = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t i = b + threadIdx.x * kPer + j;
            v[j] = i < nt ? row[i] : 0u;
            loc += v[j];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl(loc, s_w, tot);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t i = b + threadIdx.x * kPer + j;
            if (i < nt) row[i] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) C.digit_total[d] = carry;
}

template <typename K, int ITEMS>
__device__ void radix_down(const Ctx& C, uint32_t pass, uint32_t tile, char* smem) {
    constexpr int KT = kBlock * ITEMS;
    BatchState* bs = C.bs;
    const uint32_t n = n_keys(C), nt = n_sort_tiles_real<ITEMS>(C);
    const uint32_t bits = bs->pass_bits[pass], shift = bs->pass_shift[pass], D = 1u << bits;
    const K* kin = reinterpret_cast<const K*>((pass & 1) ? C.keysB : C.keysA);
    const uint32_t* vin = (pass & 1) ? C.valsB : C.valsA;
    K* kout = reinterpret_cast<K*>((pass & 1) ? C.keysA : C.keysB);
    uint32_t* vout = (pass & 1) ? C.valsA : C.valsB;

    K* s_key = reinterpret_cast<K*>(smem);                              // [KT]
    uint32_t* s_val = reinterpret_cast<uint32_t*>(s_key + KT);          // [KT]
    const uint32_t Dm = 1u << C.hdr->max_radix_bits;                    // widest digit
    uint32_t* s_wc = s_val + KT;                                        // [4][Dm] per-wave counts
    uint32_t* s_doff = s_wc + 4 * Dm;                                   // [Dm] tile digit offsets
    uint32_t* s_gb = s_doff + Dm;                                       // [Dm] global base
    uint32_t* s_w = s_gb + Dm;                                          // [8]
    uint32_t* s_cam = s_w + 8;                                          // [n_cams] pix_off
    const uint32_t tid = threadIdx.x, w = tid / kWave, l = lane_id();
    const uint32_t nc = C.hdr->n_cams;
    const bool last = pass + 1 == bs->npass && !(C.hdr->prm.flags & 1u);
    // issue this tile's key and id loads first: their latency overlaps the scans below
    const uint32_t t0 = tile * KT + w * (ITEMS * kWave);
    K key[ITEMS];
    uint32_t val[ITEMS], rank[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = t0 + (uint32_t)i * kWave + l;
        const bool in = idx < n;
        key[i] = in ? kin[idx] : (K)0;
        val[i] = in ? vin[idx] : 0u;
    }
    if (last)
        for (uint32_t i = tid; i < nc; i += kBlock) s_cam[i] = C.camlite[i].pix_off;
    for (uint32_t i = tid; i < 4 * D; i += kBlock) s_wc[i] = 0;
    // digit starts (an exclusive scan of the digit totals, done in every workgroup: D values
    // from L2, cheaper than ordering a separate scan after all column scans) plus this
    // tile's offset within each digit (its row was scanned over the tiles)
    for (uint32_t d = tid; d < D; d += kBlock) s_gb[d] = C.digit_total[d];
    __syncthreads();
    (void)lds_excl_scan(s_gb, D, s_w);
    for (uint32_t d = tid; d < D; d += kBlock) s_gb[d] += C.digit_hist[(uint64_t)d * nt + tile];

    const uint64_t lt = (l == 0) ? 0ull : ((~0ull) >> (64 - l));
    uint32_t* wc = s_wc + w * D;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = t0 + (uint32_t)i * kWave + l;
        const bool in = idx < n;
        const uint32_t dg = (uint32_t)(key[i] >> shift) & (D - 1);
        const uint64_t peers = match_peers(dg, in, bits);
        const uint32_t before = wc[dg];
        const uint32_t lower = (uint32_t)__popcll(peers & lt);
        rank[i] = before + lower;
        __builtin_amdgcn_wave_barrier();
        if (in && lower == 0) wc[dg] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per-digit tile totals (into s_doff) and per-wave offsets inside each digit
    for (uint32_t d = tid; d < D; d += kBlock) {
        uint32_t acc = 0;
        for (int ww = 0; ww < 4; ++ww) {
            const uint32_t c = s_wc[ww * D + d];
            s_wc[ww * D + d] = acc;
            acc += c;
        }
        s_doff[d] = acc;
    }
    __syncthreads();
    (void)lds_excl_scan(s_doff, D, s_w);
    for (uint32_t d = tid; d < D; d += kBlock) s_gb[d] -= s_doff[d];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = t0 + (uint32_t)i * kWave + l;
        if (idx >= n) continue;
        const uint32_t dg = (uint32_t)(key[i] >> shift) & (D - 1);
        const uint32_t pos = s_doff[dg] + s_wc[w * D + dg] + rank[i];
        s_key[pos] = key[i];
        s_val[pos] = val[i];
    }
    __syncthreads();
    const uint32_t cnt = min((uint32_t)KT, n - tile * KT);
    for (uint32_t s = tid; s < cnt; s += kBlock) {
        const K kk = s_key[s];
        const uint32_t dg = (uint32_t)(kk >> shift) & (D - 1);
        const uint32_t dst = s_gb[dg] + s;
        if (dst >= n) { raise_error(bs, kErrBounds); continue; }
        const uint32_t v = s_val[s];
        kout[dst] = kk;
        vout[dst] = v;
        if (last) {
            // the per-cell phase ranks members by confidence: hand it over in sorted order
            const CamLite& cl = C.camlite[last_le(s_cam, (int)nc, v)];
            C.conf_sorted[dst] = __float_as_uint(glob(cl.conf)[v - cl.pix_off]);
        }
    }
}

template <int ITEMS>
__device__ __forceinline__ void ph_radix_down(const Ctx& C, uint32_t pass, uint32_t tile, char* smem) {
    BatchState* bs = C.bs;
    if ((C.hdr->prm.flags & 4u) || pass >= bs->npass) return;
    if (tile >= n_sort_tiles_real<ITEMS>(C)) return;
    if (bs->key64) radix_down<uint64_t, ITEMS>(C, pass, tile, smem);
    else radix_down<uint32_t, ITEMS>(C, pass, tile, smem);
}

// final (sorted) buffers
__device__ __forceinline__ const uint32_t* sorted_vals(const Ctx& C) {
    return (C.bs->npass & 1) ? C.valsB : C.valsA;
}
__device__ __forceinline__ uint64_t sorted_key(const Ctx& C, uint32_t i) {
    return load_key(C, C.bs->npass & 1, C.bs->key64, i);
}

// ---------------------------------------------------------------- cell heads
// Cells are runs of equal keys in sorted order: count the run heads per tile, scan, write
// each cell's first position, and record where each frame's cells begin.

// Thread t of a sort tile takes the tile's ITEMS consecutive sorted keys from
// first = tile * 256 ITEMS + t ITEMS (32-bit keys read as 16-byte vectors).  Bit i of the
// returned flags: key first + i starts a run (it is the first key, or differs from the key
// before it).  The keys (k) and the key before them (prev) are returned for the head
// writer's frame test.
template <int ITEMS>
__device__ __forceinline__ uint32_t head_flags(const Ctx& C, uint32_t tile, uint32_t n,
                                               uint32_t& first, uint64_t (&k)[ITEMS],
                                               uint64_t& prev) {
    first = tile * (kBlock * ITEMS) + threadIdx.x * ITEMS;
    if (first >= n) return 0u;
    const bool key64 = C.bs->key64, from_b = C.bs->npass & 1;
    prev = first == 0 ? 0ull : load_key(C, from_b, key64, first - 1);
    if (!key64 && first + ITEMS <= n) {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        const u4* kp = reinterpret_cast<const u4*>(
            reinterpret_cast<const uint32_t*>(from_b ? C.keysB : C.keysA) + first);
#pragma unroll
        for (int q = 0; q < ITEMS / 4; ++q) {
            const u4 v = glob(kp)[q];
            k[4 * q] = v.x; k[4 * q + 1] = v.y; k[4 * q + 2] = v.z; k[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            k[i] = first + (uint32_t)i < n ? load_key(C, from_b, key64, first + i) : 0ull;
    }
    uint32_t flags = first == 0 ? 1u : (k[0] != prev ? 1u : 0u);
#pragma unroll
    for (int i = 1; i < ITEMS; ++i)
        if (first + (uint32_t)i < n && k[i] != k[i - 1]) flags |= 1u << i;
    return flags;
}

template <int ITEMS>
__device__ __forceinline__ void ph_head_count(const Ctx& C, uint32_t tile, char* smem) {
    if (C.hdr->prm.flags & 4u) return;
    const uint32_t n = n_keys(C);
    if (tile >= n_sort_tiles_real<ITEMS>(C)) return;
    uint32_t first;
    uint64_t k[ITEMS], prev;
    const uint32_t c = (uint32_t)__popc(head_flags<ITEMS>(C, tile, n, first, k, prev));
    const uint32_t tot = block_sum(c, reinterpret_cast<uint32_t*>(smem));
    if (threadIdx.x == 0) C.head_cnt[tile] = tot;
}

template <int ITEMS>
__device__ __forceinline__ void ph_head_scan(const Ctx& C, uint32_t, char* smem) {
    if (C.hdr->prm.flags & 4u) return;
    const uint32_t n = n_keys(C), nt = n_sort_tiles_real<ITEMS>(C);
    uint32_t* s_w = reinterpret_cast<uint32_t*>(smem);
    const bool one_step = nt <= (uint32_t)(kBlock * kRowScanPer);
    uint32_t carry = one_step ? row_scan_one_step(C.head_cnt, nt, s_w) : 0u;
    constexpr int kPer = 8;                  // consecutive tiles per thread per step
    for (uint32_t b = one_step ? nt : 0u; b < nt; b += kBlock * kPer) {
        uint32_t v[kPer], sum = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t i = b + threadIdx.x * kPer + j;
            v[j] = i < nt ? C.head_cnt[i] : 0u;
            sum += v[j];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl(sum, s_w, tot);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t i = b + threadIdx.x * kPer + j;
            if (i < nt) C.head_cnt[i] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        C.bs->S_tot = carry;
        if (carry <= C.P_cap) C.cell_start[carry] = n;
    }
}

// frame of a dense key: frames own disjoint ascending key ranges starting at fine_begin
__device__ __forceinline__ int frame_of_key(const uint64_t* fbeg, int nf, uint64_t k) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fbeg[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int ITEMS>
__device__ __forceinline__ void ph_head_write(const Ctx& C, uint32_t tile, char* smem) {
    const CallHdr& H = *C.hdr;
    if (H.prm.flags & 4u) return;
    const uint32_t n = n_keys(C);
    if (tile >= n_sort_tiles_real<ITEMS>(C)) return;
    uint64_t* s_fbeg = reinterpret_cast<uint64_t*>(smem);               // [F]
    uint32_t* s_w = reinterpret_cast<uint32_t*>(s_fbeg + kMaxFrames);   // [4]
    const uint32_t nf = H.n_frames;
    for (uint32_t f = threadIdx.x; f < nf; f += kBlock) s_fbeg[f] = C.fs[f].fine_begin;
    uint32_t first;
    uint64_t k[ITEMS], prev;
    const uint32_t flags = head_flags<ITEMS>(C, tile, n, first, k, prev);
    uint32_t tot;
    // the tile's cells are numbered in key order: thread order, then bit order
    uint32_t pos = C.head_cnt[tile] + block_excl((uint32_t)__popc(flags), s_w, tot);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (!(flags >> i & 1u)) continue;
        const uint32_t idx = first + (uint32_t)i;
        if (pos < C.P_cap) C.cell_start[pos] = idx; else raise_error(C.bs, kErrBounds);
        // the first cell of a frame: the previous element belongs to another frame
        const int f = frame_of_key(s_fbeg, (int)nf, k[i]);
        if (idx == 0 || frame_of_key(s_fbeg, (int)nf, i == 0 ? prev : k[i - 1]) != f) {
            C.fs[f].cell_begin = pos;
            C.fs[f].has_cells = 1;
        }
        ++pos;
    }
}

// ---------------------------------------------------------------- cell helpers

// A member of a cell for the full-order ranking; its pixel id and position are fetched
// only when needed.
struct Cand {
    float C;
    uint32_t k;      // sorted position
    uint32_t id;     // batch pixel id (valid when st >= 1)
    int cam;         // camera (valid when st >= 1)
    int st;          // 0: C only, 1: + id and camera, 2: + position
    Pt p;
};

// Per-wave staging of the per-cell phase: 64 cells and their up to 192 representatives.
constexpr int kStageCells = 64;
struct WaveStage {
    uint32_t start[kStageCells];
    uint32_t end[kStageCells];               // start == end: no output for this slot
    uint32_t sid[3 * kStageCells];           // representative: sorted position, then pixel id
    float sC[3 * kStageCells];
    float px[3 * kStageCells], py[3 * kStageCells], pz[3 * kStageCells];
    uint32_t rgb[3 * kStageCells];
    uint32_t ex_lo[3 * kStageCells], ex_hi[3 * kStageCells];   // -ln V as a double
    uint8_t list[3 * kStageCells];           // compacted representative slots
    uint8_t bad[kStageCells];
};
constexpr int kCellsStageBytes = (kBlock / 64) * (int)sizeof(WaveStage);

// LDS of the per-cell phase: this header, then the cameras' pixel offsets, then (when few
// enough) the camera records, then one stage per wave.
struct CellsShared {
    uint32_t fpix[kMaxFrames];                  // frame pix_begin
    uint32_t key_begin[kMaxFrames];             // frame's first sorted/compacted position
    uint32_t cell_begin[kMaxFrames];            // frame's first global cell
    uint32_t rcount[kMaxFrames];                // representatives per frame (this workgroup)
};

struct CellsLayout {
    uint32_t cam_pix, cams, frames, grids, stage, total;   // byte offsets, total bytes
};
__host__ __device__ inline CellsLayout cells_layout(uint32_t ncams, bool lds_cams,
                                                    uint32_t nframes) {
    CellsLayout l;
    l.cam_pix = (uint32_t)sizeof(CellsShared);
    l.cams = (l.cam_pix + 4 * ncams + 15u) & ~15u;
    l.frames = (l.cams + (lds_cams ? ncams * (uint32_t)sizeof(CamLite) : 0u) + 15u) & ~15u;
    l.grids = (l.frames + nframes * (uint32_t)sizeof(DevFrame) + 15u) & ~15u;
    l.stage = (l.grids + nframes * (uint32_t)sizeof(FrameGrid) + 15u) & ~15u;
    l.total = l.stage + (uint32_t)kCellsStageBytes;
    return l;
}

struct CellCtx {
    const Ctx& C;
    const CamLite* cams;      // LDS copy when the batch has few cameras, else global
    const uint32_t* cam_pix;  // LDS
    const uint32_t* vals;
    int nc;
};

__device__ __forceinline__ void ensure_id(const CellCtx& X, Cand& a) {
    if (a.st >= 1) return;
    a.id = glob(X.vals)[a.k];
    a.cam = last_le(X.cam_pix, X.nc, a.id);
    a.st = 1;
}

// (x, y) of pixel `loc` of a camera: a float estimate of loc / W, then exact correction.
// 32-bit integers suffice: loc < W H <= 2^28 and the estimate is within one row of y.
template <typename Cam>
__device__ __forceinline__ void pixel_xy(const Cam& cm, uint32_t loc, uint32_t& x, uint32_t& y) {
    const int32_t W = cm.W;
    int32_t yy = (int32_t)((float)loc * cm.invW);
    int32_t r = (int32_t)loc - yy * W;
    while (r < 0) { --yy; r += W; }
    while (r >= W) { ++yy; r -= W; }
    y = (uint32_t)yy;
    x = (uint32_t)r;
}

__device__ __forceinline__ void ensure_p(const CellCtx& X, Cand& a) {
    if (a.st >= 2) return;
    ensure_id(X, a);
    const CamLite& cm = X.cams[a.cam];
    const uint32_t loc = a.id - cm.pix_off;
    uint32_t x, y;
    pixel_xy(cm, loc, x, y);
    a.p = backproject_ray(cm, ((float)x - cm.cx) / cm.fx, ((float)y - cm.cy) / cm.fy,
                          glob(cm.depth)[loc]);
    a.st = 2;
}

// strict "a ranks before b": C descending, then x, y, z ascending, then pixel id
__device__ __forceinline__ bool rank_before(const CellCtx& X, Cand& a, Cand& b) {
    if (a.C != b.C) return a.C > b.C;
    ensure_p(X, a);
    ensure_p(X, b);
    if (a.p.x != b.p.x) return a.p.x < b.p.x;
    if (a.p.y != b.p.y) return a.p.y < b.p.y;
    if (a.p.z != b.p.z) return a.p.z < b.p.z;
    return a.id < b.id;
}

// Insert c into the ascending list s of the N smallest keys seen (an empty slot holds the
// largest key).  Every comparison is against the old list, which is sorted, so slot q
// takes s[q-1] when c goes before it, else c when c goes before s[q], else keeps s[q]:
// N independent compares instead of a chain of minimum/maximum pairs.
template <int N>
__device__ __forceinline__ void insert_sorted(uint64_t (&s)[N], uint64_t c) {
    bool b[N];
#pragma unroll
    for (int q = 0; q < N; ++q) b[q] = c < s[q];
#pragma unroll
    for (int q = N - 1; q > 0; --q) s[q] = b[q - 1] ? s[q - 1] : (b[q] ? c : s[q]);
    s[0] = b[0] ? c : s[0];
}

// -ln V of representative (camera ri, point p): Eq. 4-7 over the first K-1 views by
// distance.  KV >= K - 1 is the compile-time size of the kept list.  The field-of-view
// classes of the point's coarse cell (in_all, partial: bits over the frame's cameras) say
// which cameras see the whole cell, which see none of it and which need the exact test of
// this point; only the last take it.  A visible camera becomes the 64-bit key (bits of the
// squared distance, camera rank, camera index): the bits of a non-negative float order
// like its value and ranks are unique within a frame, so keys order candidates by
// (distance, rank).  A branch-free insertion keeps the KV smallest keys sorted.  A camera
// no lane of the wave can see is skipped as a whole.
template <int KV>
__device__ __forceinline__ double neg_log_v(const CamLite* cams, const float* raytab,
                                            uint32_t own_bit, const Pt& p,
                                            uint32_t fcam0, uint32_t fcams, uint64_t in_all,
                                            uint64_t partial, const DevParams& P) {
    const int keep = (P.K < (int)fcams ? P.K : (int)fcams) - 1;
    if (keep <= 0) return 0.0;
    constexpr uint64_t kNone = ~0ull;
    uint64_t best[KV];
#pragma unroll
    for (int q = 0; q < KV; ++q) best[q] = kNone;
    const uint64_t cand = (in_all | partial) & ~(1ull << own_bit);
    for (uint32_t jj = 0; jj < fcams; ++jj) {
        const bool c_j = (cand >> jj) & 1ull;
        if (__ballot(c_j) == 0ull) continue;          // no lane can see this camera
        const uint32_t j = fcam0 + jj;
        const CamLite& cj = cams[j];
        bool vis = c_j && ((in_all >> jj) & 1ull);
        const bool part = c_j && ((partial >> jj) & 1ull);
        if (__ballot(part) != 0ull) {
            if (part) vis = in_view_fast(cj, p);
        }
        const float dx = p.x - cj.c[0], dy = p.y - cj.c[1], dz = p.z - cj.c[2];
        const float d2 = (dx * dx + dy * dy) + dz * dz;
        const uint64_t c = vis ? ((uint64_t)__float_as_uint(d2) << 32 | (uint64_t)cj.rank << 16 | j)
                               : kNone;
        insert_sorted(best, c);
    }
    int nb = 0;
    int bj[KV];
#pragma unroll
    for (int q = 0; q < KV; ++q) {
        bj[q] = (int)(best[q] & 0xFFFFu);
        if (q < keep && best[q] != kNone) nb = q + 1;
    }
    // pixels of the kept views (the camera-frame point is recomputed: cheaper than carrying
    // it), then their depths and pixel rays as independent gathers
    int bx[KV], by[KV];
    float dv[KV], rxv[KV], ryv[KV];
#pragma unroll
    for (int q = 0; q < KV; ++q) {
        dv[q] = rxv[q] = ryv[q] = 0.0f;
        bx[q] = by[q] = 0;
        if (q < nb) {
            const CamLite& cj = cams[bj[q]];
            const float X = ((cj.R[0] * p.x + cj.R[1] * p.y) + cj.R[2] * p.z) + cj.t[0];
            const float Y = ((cj.R[3] * p.x + cj.R[4] * p.y) + cj.R[5] * p.z) + cj.t[1];
            const float Z = ((cj.R[6] * p.x + cj.R[7] * p.y) + cj.R[8] * p.z) + cj.t[2];
            exact_pixel(cj, X, Y, Z, bx[q], by[q]);
            dv[q] = glob(cj.depth)[(uint32_t)by[q] * (uint32_t)cj.W + (uint32_t)bx[q]];
            const float* rt = raytab + cj.tab_off;
            rxv[q] = glob(rt)[bx[q]];
            ryv[q] = glob(rt + cj.W)[by[q]];
        }
    }
    double s = 0.0;
    int m = 0;
#pragma unroll
    for (int q = 0; q < KV; ++q) {
        if (q >= nb) continue;
        const float d = dv[q];
        if (!(__builtin_isfinite(d) && d > 0.0f)) continue;
        const CamLite& cj = cams[bj[q]];
        // the ray of pixel (bx, by) from the camera's ray tables (the IEEE quotients
        // (x - cx)/fx and (y - cy)/fy), loaded beside the depth: cheaper than two divisions
        const Pt Q = backproject_ray(cj, rxv[q], ryv[q], d);
        // the differences of two floats and their squares are exact in double
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

// ---------------------------------------------------------------- quad exchange
// Four consecutive lanes of a wave work on one cell.  DPP quad permutations move values
// between them; every use sits where all four lanes of the quad are active.
template <int CTRL>
__device__ __forceinline__ uint32_t qmov(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float qmovf(float v) {
    return __uint_as_float(qmov<CTRL>(__float_as_uint(v)));
}
constexpr int kQuadXor1 = 0xB1;                 // lanes [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;                 // lanes [2, 3, 0, 1]
template <int R> struct QuadBcast { static constexpr int ctrl = R * 0x55; };   // [R, R, R, R]

// insert c into the sorted list of the best n <= 3 members (full order)
__device__ __forceinline__ void top3_insert(const CellCtx& X, Cand* rep, int& n, Cand& c) {
    if (n == 3 && !rank_before(X, c, rep[2])) return;
    if (n < 1 || rank_before(X, c, rep[0])) {
        rep[2] = rep[1]; rep[1] = rep[0]; rep[0] = c;
    } else if (n < 2 || rank_before(X, c, rep[1])) {
        rep[2] = rep[1]; rep[1] = c;
    } else {
        rep[2] = c;
    }
    if (n < 3) ++n;
}

// Confidence as an order-preserving unsigned value (-0 taken as +0): a larger confidence
// gives a larger value, and none gives 0 (that would be a negative NaN, which fails the
// gate).
__device__ __forceinline__ uint32_t conf_bits(float c) { return f2o(c + 0.0f); }

__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
    return max(min(a, b), min(max(a, b), c));
}

// The three largest confidence values t0 >= t1 >= t2 of a set (0 = empty slot) and the
// sorted positions k0, k1, k2 of the members that hold them (kPad for an empty slot), kept
// by a three-instruction insertion network plus one select per position.  `tie` is set
// whenever a value equal to a kept one is met: only then can the position / pixel
// tie-break of the full order change the choice or the order of the three, and the caller
// ranks that cell again in full.  Without a tie each of the three values belongs to
// exactly one member, whose position is the one kept beside it.
struct Top3p {
    uint32_t t0, t1, t2, k0, k1, k2;
    bool tie;
};
__device__ __forceinline__ void top3p_push(Top3p& t, uint32_t v, uint32_t k) {
    t.tie |= (v != 0u) & ((v == t.t0) | (v == t.t1) | (v == t.t2));
    const bool g0 = v > t.t0, g1 = v > t.t1, g2 = v > t.t2;
    const uint32_t nk0 = g0 ? k : t.k0;
    const uint32_t nk1 = g0 ? t.k0 : (g1 ? k : t.k1);
    const uint32_t nk2 = g1 ? t.k1 : (g2 ? k : t.k2);
    const uint32_t n0 = max(t.t0, v), n1 = med3u(t.t0, t.t1, v), n2 = med3u(t.t1, t.t2, v);
    t.t0 = n0;
    t.t1 = n1;
    t.t2 = n2;
    t.k0 = nk0;
    t.k1 = nk1;
    t.k2 = nk2;
}
// merge the partner lane's three (disjoint members) into this lane's
template <int CTRL>
__device__ __forceinline__ void top3p_merge(Top3p& t) {
    const uint32_t a = qmov<CTRL>(t.t0), b = qmov<CTRL>(t.t1), c = qmov<CTRL>(t.t2);
    const uint32_t ka = qmov<CTRL>(t.k0), kb = qmov<CTRL>(t.k1), kc = qmov<CTRL>(t.k2);
    t.tie |= qmov<CTRL>(t.tie ? 1u : 0u) != 0u;
    top3p_push(t, a, ka);
    top3p_push(t, b, kb);
    top3p_push(t, c, kc);
}

// Output of one cell from its representatives' values: joint weights w = C V (Eq. 10) and
// the normalised weighted mean (Eq. 11), taken as a softmax of a = ln C - ln V^-1 so that
// no weight underflows; the output weight is the mean of the w.  The exponents are formed
// in double and their exponentials (all <= 1) taken in float32.
__device__ __forceinline__ void emit_cell(const DevFrame& fr, uint32_t o, int nrep,
                                          const float* Cr, const Pt* pr, const double* expo,
                                          const uint32_t* rgb3, const uint32_t* idr,
                                          uint32_t nmem) {
    constexpr double kLog2e = 1.4426950408889634;
    double a[3], amax = -INFINITY;
    bool nan = false;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        a[r] = r < nrep ? (double)logf(Cr[r]) - expo[r] : -INFINITY;
        nan |= a[r] != a[r];
        amax = a[r] > amax ? a[r] : amax;
    }
    if (nan) amax = __longlong_as_double(0x7FF8000000000000ll);   // as the mean of NaNs
    float e[3], se = 0.0f, wsum = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        e[r] = r < nrep ? exp2f((float)((a[r] - amax) * kLog2e)) : 0.0f;
        se += e[r];
        wsum += r < nrep ? Cr[r] * exp2f((float)(-expo[r] * kLog2e)) : 0.0f;
    }
    float x = 0.0f, y = 0.0f, z = 0.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        if (r >= nrep) continue;
        const float pi = e[r] / se;
        x += pi * pr[r].x;
        y += pi * pr[r].y;
        z += pi * pr[r].z;
        cr += pi * (float)(rgb3[r] & 0xFFu);
        cg += pi * (float)(rgb3[r] >> 8 & 0xFFu);
        cb += pi * (float)(rgb3[r] >> 16 & 0xFFu);
    }
    glob(fr.xyz)[(uint64_t)o * 3 + 0] = x;
    glob(fr.xyz)[(uint64_t)o * 3 + 1] = y;
    glob(fr.xyz)[(uint64_t)o * 3 + 2] = z;
    glob(fr.weight)[o] = wsum / (float)nrep;
    if (fr.rgb != nullptr && fr.has_rgb) {
        const float v[3] = {cr, cg, cb};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float t = rintf(v[k]);
            t = t > 0.0f ? (t > 255.0f ? 255.0f : t) : 0.0f;     // NaN -> 0
            glob(fr.rgb)[(uint64_t)o * 3 + k] = (uint8_t)t;
        }
    }
    if (fr.n_members) glob(fr.n_members)[o] = nmem;
    if (fr.reps) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
            glob(fr.reps)[(uint64_t)o * 3 + r] = r < nrep ? idr[r] - fr.pix_begin : kPad;
    }
}

// LDS written by some lanes of a wave and read by others: order the wave's accesses
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- phase: cells
// Top-3 representatives (Sec. II.5(2)a), local views and consistency (II.5(2)b, Eq. 4-7),
// joint weight and fusion (Eq. 10-11), output.  A wave takes 64 cells at a time through
// three stages that each keep all 64 lanes busy, handing over through its own LDS stage:
//   A  cells of at most three members: one lane per cell orders their confidences; larger
//      cells (and ties): four lanes per cell, each ranking every fourth member, the lists
//      merged across the quad, 16 cells at a time;
//   B  the representatives, compacted, one per lane: back-projection, local views, -ln V;
//   C  one lane per cell: key, joint weights, fused point, outputs.
// Waves walk groups of 64 cells; the workgroups of one XCD (dispatched round-robin over
// the eight) share one contiguous range of cells, so nearby cells, which see nearby
// pixels, meet in the same L2.

template <int KV, bool LDS_CAMS>
__device__ __forceinline__ void ph_cells(const Ctx& C, uint32_t item, char* smem) {
    const CallHdr& H = *C.hdr;
    const DevParams& P = H.prm;
    BatchState* bs = C.bs;
    CellsShared& sh = *reinterpret_cast<CellsShared*>(smem);
    const CellsLayout lay = cells_layout(H.n_cams, LDS_CAMS, H.n_frames);
    uint32_t* s_cam_pix = reinterpret_cast<uint32_t*>(smem + lay.cam_pix);
    CamLite* s_cams = reinterpret_cast<CamLite*>(smem + lay.cams);
    const uint32_t nf = H.n_frames, nc = H.n_cams;
    const bool no_sa = P.flags & 4u, no_mf = P.flags & 1u, no_dc = P.flags & 2u;
    for (uint32_t i = threadIdx.x; i < nc; i += kBlock) {
        s_cam_pix[i] = C.camlite[i].pix_off;
        if (LDS_CAMS) s_cams[i] = C.camlite[i];
    }
    // the frames' records and coarse grids, read by every cell: from LDS, not through
    // dependent global loads
    DevFrame* s_frames = reinterpret_cast<DevFrame*>(smem + lay.frames);
    FrameGrid* s_grids = reinterpret_cast<FrameGrid*>(smem + lay.grids);
    for (uint32_t f = threadIdx.x; f < nf; f += kBlock) {
        sh.fpix[f] = C.frames[f].pix_begin;
        sh.key_begin[f] = C.fs[f].key_begin;
        sh.cell_begin[f] = no_sa ? C.fs[f].key_begin : C.fs[f].cell_begin;
        sh.rcount[f] = 0;
        s_frames[f] = C.frames[f];
        frame_grid(C.fs[f], P, s_grids[f]);
    }
    __syncthreads();
    const uint32_t M_tot = n_keys(C);
    const uint32_t S = min(no_sa ? bs->M_tot : bs->S_tot, M_tot);
    const uint32_t n_items = H.n_cell_items;
    const uint32_t* vals = no_sa ? C.valsA : sorted_vals(C);
    // one source per instantiation, so LDS reads compile to ds_read (a pointer that may be
    // either LDS or global would make every camera read a flat access that waits for all
    // outstanding global loads)
    const CamLite* cams = LDS_CAMS ? s_cams : C.camlite;
    const CellCtx X{C, cams, s_cam_pix, vals, (int)nc};
    // confidences in sorted order come from the last radix pass (none ran: gather them)
    const bool have_cs = !no_sa && !no_mf && bs->npass > 0;
    const uint32_t G3 = (uint32_t)(P.G * P.G * P.G);
    const bool fr_mids_any = H.any_mids != 0;
    const uint32_t lane = threadIdx.x & 63u, q = lane & 3u;
    const uint32_t wpb = kBlock / 64, wave = threadIdx.x >> 6;
    WaveStage& st = reinterpret_cast<WaveStage*>(smem + lay.stage)[wave];
    const uint32_t nx = min(8u, n_items), xcd = item % nx, li = item / nx;
    const uint32_t n_local = (n_items - xcd + nx - 1) / nx;
    const uint32_t r0 = (uint32_t)((uint64_t)S * xcd / nx);
    const uint32_t r1 = (uint32_t)((uint64_t)S * (xcd + 1) / nx);
    for (uint32_t g0 = r0 + (li * wpb + wave) * kStageCells; g0 < r1;
         g0 += n_local * wpb * kStageCells) {
        // member ranges of all 64 cells at once (lane = cell).  A cell of at most three
        // members needs no selection: its lane orders their confidences; a tie among them
        // goes to the quads, which settle it in the full order.  The other cells are listed
        // for the quads.
        bool big = false;
        {
            const uint32_t s = g0 + lane;
            uint32_t a = 0, b = 0;
            if (s < r1) {
                if (no_sa) { a = s; b = s + 1; }
                else { a = glob(C.cell_start)[s]; b = glob(C.cell_start)[s + 1]; }
            }
            bool small = false;
            if (s < r1 && have_cs && a < b && b <= M_tot && b - a <= 3u) {
                const uint32_t n = b - a;
                uint32_t v0 = conf_bits(__uint_as_float(glob(C.conf_sorted)[a]));
                uint32_t v1 = n > 1 ? conf_bits(__uint_as_float(glob(C.conf_sorted)[a + 1])) : 0u;
                uint32_t v2 = n > 2 ? conf_bits(__uint_as_float(glob(C.conf_sorted)[a + 2])) : 0u;
                uint32_t k0 = a, k1 = a + 1, k2 = a + 2;
                // three-element sorting network, descending value; positions ride along
                auto cswap = [](uint32_t& va, uint32_t& ka, uint32_t& vb, uint32_t& kb) {
                    const bool sw = vb > va;
                    const uint32_t tv = sw ? vb : va, tk = sw ? kb : ka;
                    vb = sw ? va : vb;
                    kb = sw ? ka : kb;
                    va = tv;
                    ka = tk;
                };
                cswap(v0, k0, v1, k1);
                cswap(v1, k1, v2, k2);
                cswap(v0, k0, v1, k1);
                small = !((n > 1 && v0 == v1) || (n > 2 && v1 == v2));
                if (small) {
                    st.sid[lane * 3 + 0] = k0;
                    st.sC[lane * 3 + 0] = o2f(v0);
                    if (n > 1) { st.sid[lane * 3 + 1] = k1; st.sC[lane * 3 + 1] = o2f(v1); }
                    if (n > 2) { st.sid[lane * 3 + 2] = k2; st.sC[lane * 3 + 2] = o2f(v2); }
                    if (fr_mids_any) {
                        const int f = last_le(sh.fpix, (int)nf, glob(vals)[a]);
                        const DevFrame& fr = s_frames[f];
                        if (fr.mids) {
                            for (uint32_t k = a; k < b; ++k) {
                                const uint32_t mo = k - sh.key_begin[f];
                                if (mo < fr.member_capacity)
                                    glob(fr.mids)[mo] = glob(vals)[k] - fr.pix_begin;
                            }
                        }
                    }
                }
            }
            big = s < r1 && !small;
            st.start[lane] = a;
            st.end[lane] = b;
            st.bad[lane] = 0;
        }
        const uint64_t bigm = __ballot(big);
        const uint32_t nbig = (uint32_t)__popcll(bigm);
        if (big) {
            const uint64_t below = lane == 0u ? 0ull : (~0ull >> (64u - lane));
            st.list[__popcll(bigm & below)] = (uint8_t)lane;
        }
        wave_sync();
        // ---- A: top-3 of the listed cells, 16 per pass, four lanes per cell
        for (uint32_t sub = 0; sub < nbig; sub += 16u) {
            const uint32_t jj = sub + (lane >> 2);
            const bool have = jj < nbig;
            const uint32_t j = have ? (uint32_t)st.list[jj] : 0u;
            const uint32_t s = g0 + j;
            uint32_t start = 0, end = 0;
            bool ok = have && s < r1;
            if (ok) {
                start = st.start[j];
                end = st.end[j];
                if (end > M_tot || start >= end) {
                    if (q == 0) raise_error(bs, kErrBounds);
                    ok = false;
                }
            }
            if (ok) {
                // this lane's members start + q, start + q + 4, ...: confidences of 4 of
                // them are loaded together (most cells give a lane one or two members),
                // then ranked by value with their positions carried along; the positions
                // are the representatives unless a tie was seen
                auto conf_at = [&](uint32_t k) -> float {
                    if (have_cs) return __uint_as_float(glob(C.conf_sorted)[k]);
                    const uint32_t id = glob(vals)[k];
                    const CamLite& cm = cams[last_le(s_cam_pix, (int)nc, id)];
                    return glob(cm.conf)[id - cm.pix_off];
                };
                Top3p t{0u, 0u, 0u, kPad, kPad, kPad, no_mf};   // all confidences 1: full order
                if (!no_mf) {
                    for (uint32_t k0 = start + q; k0 < end; k0 += 16u) {
                        float cv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const uint32_t k = k0 + 4u * u;
                            cv[u] = k < end ? conf_at(k) : 0.0f;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const uint32_t k = k0 + 4u * u;
                            if (k < end) top3p_push(t, conf_bits(cv[u]), k);
                        }
                    }
                }
                top3p_merge<kQuadXor1>(t);
                top3p_merge<kQuadXor2>(t);
                const int nrep = (int)min(3u, end - start);
                uint32_t kr0 = kPad, kr1 = kPad, kr2 = kPad;
                float cr0 = o2f(t.t0), cr1 = o2f(t.t1), cr2 = o2f(t.t2);
                if (!t.tie) {
                    kr0 = t.k0;
                    kr1 = t.k1;
                    kr2 = t.k2;
                } else {
                    // equal confidences among the best: lane 0 ranks the whole cell in the
                    // full order (confidence, then position, then pixel id)
                    if (q == 0u) {
                        Cand rep[3];
                        int n = 0;
#pragma unroll 1
                        for (uint32_t k = start; k < end; ++k) {
                            Cand c;
                            c.k = k;
                            c.st = 0;
                            c.id = 0;
                            c.cam = 0;
                            c.C = no_mf ? 1.0f : conf_at(k);
                            top3_insert(X, rep, n, c);
                        }
                        kr0 = rep[0].k; cr0 = rep[0].C;
                        kr1 = n > 1 ? rep[1].k : 0u; cr1 = n > 1 ? rep[1].C : 0.0f;
                        kr2 = n > 2 ? rep[2].k : 0u; cr2 = n > 2 ? rep[2].C : 0.0f;
                    }
                    kr0 = qmov<QuadBcast<0>::ctrl>(kr0);
                    kr1 = qmov<QuadBcast<0>::ctrl>(kr1);
                    kr2 = qmov<QuadBcast<0>::ctrl>(kr2);
                    cr0 = qmovf<QuadBcast<0>::ctrl>(cr0);
                    cr1 = qmovf<QuadBcast<0>::ctrl>(cr1);
                    cr2 = qmovf<QuadBcast<0>::ctrl>(cr2);
                }
                if ((int)q < nrep) {
                    const uint32_t kq = q == 1u ? kr1 : (q == 2u ? kr2 : kr0);
                    if (kq >= end) {                  // every value is some member's
                        raise_error(bs, kErrBounds);
                        st.bad[j] = 1;
                    }
                    st.sid[j * 3 + q] = kq < end ? kq : start;
                    st.sC[j * 3 + q] = q == 1u ? cr1 : (q == 2u ? cr2 : cr0);
                }
                if (fr_mids_any) {
                    const int f = last_le(sh.fpix, (int)nf, glob(vals)[start]);
                    const DevFrame& fr = s_frames[f];
                    if (fr.mids) {
                        for (uint32_t k = start + q; k < end; k += 4u) {
                            const uint32_t mo = k - sh.key_begin[f];
                            if (mo < fr.member_capacity)
                                glob(fr.mids)[mo] = glob(vals)[k] - fr.pix_begin;
                        }
                    }
                }
            } else {
                start = end = 0;
            }
            if (have && q == 0u) {
                st.start[j] = start;
                st.end[j] = end;
            }
        }
        wave_sync();
        // ---- compaction of the representatives (lane = cell)
        const uint32_t nrep_l = st.bad[lane] ? 0u : min(3u, st.end[lane] - st.start[lane]);
        const uint32_t incl = wave_incl(nrep_l);
        const uint32_t T = __shfl(incl, 63);
        for (uint32_t r = 0; r < nrep_l; ++r) st.list[incl - nrep_l + r] = (uint8_t)(lane * 3 + r);
        wave_sync();
        // ---- B: one representative per lane
        for (uint32_t i0 = 0; i0 < T; i0 += 64u) {
            const uint32_t i = i0 + lane;
            if (i >= T) continue;
            const uint32_t slot = st.list[i];
            const uint32_t j = slot / 3u;
            Cand mine;
            mine.k = st.sid[slot];
            mine.C = st.sC[slot];
            mine.st = 0;
            mine.id = 0;
            mine.cam = 0;
            ensure_id(X, mine);
            const CamLite& cm = cams[mine.cam];
            if (mine.id >= H.P_tot || mine.id - cm.pix_off >= (uint32_t)cm.W * (uint32_t)cm.H) {
                raise_error(bs, kErrBounds);
                st.bad[j] = 1;
                continue;
            }
            ensure_p(X, mine);
            const uint32_t f = cm.frame;
            const DevFrame& fr = s_frames[f];
            double expo = 0.0;
            if (!no_dc) {
                uint64_t in_all = 0ull, partial = ~0ull;
                if (!no_sa) {
                    const CellCoord cc = coarse_cell(s_grids[f], mine.p);
                    const auto kc = glob(C.cls) + ((uint64_t)f * G3 + cc.lin);
                    in_all = kc->in_all;
                    partial = kc->partial;
                }
                expo = neg_log_v<KV>(cams, C.raytab, cm.frame_cam, mine.p, fr.cam_begin, fr.n_cams,
                                     in_all, partial, P);
            }
            uint32_t rgb3 = 0;
            if (fr.rgb != nullptr && fr.has_rgb) {
                const auto px = glob(cm.rgb + (uint64_t)(mine.id - cm.pix_off) * 3);
                rgb3 = (uint32_t)px[0] | (uint32_t)px[1] << 8 | (uint32_t)px[2] << 16;
            }
            const uint64_t eb = (uint64_t)__double_as_longlong(expo);
            st.sid[slot] = mine.id;
            st.px[slot] = mine.p.x;
            st.py[slot] = mine.p.y;
            st.pz[slot] = mine.p.z;
            st.rgb[slot] = rgb3;
            st.ex_lo[slot] = (uint32_t)eb;
            st.ex_hi[slot] = (uint32_t)(eb >> 32);
        }
        wave_sync();
        // ---- C: one cell per lane
        {
            const uint32_t j = lane, s = g0 + j;
            const uint32_t start = st.start[j], end = st.end[j];
            const int nrep = (int)min(3u, end - start);
            if (nrep > 0 && !st.bad[j]) {
                float Cr[3];
                Pt pr[3];
                double ex[3];
                uint32_t c3[3], ids[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const uint32_t sl = j * 3 + r;
                    const bool h = r < nrep;
                    Cr[r] = h ? st.sC[sl] : 0.0f;
                    pr[r] = h ? Pt{st.px[sl], st.py[sl], st.pz[sl]} : Pt{0.0f, 0.0f, 0.0f};
                    ex[r] = h ? __longlong_as_double((long long)((uint64_t)st.ex_lo[sl] |
                                                                 ((uint64_t)st.ex_hi[sl] << 32)))
                              : 0.0;
                    c3[r] = h ? st.rgb[sl] : 0u;
                    ids[r] = h ? st.sid[sl] : 0u;
                }
                const int f = last_le(sh.fpix, (int)nf, ids[0]);
                const DevFrame& fr = s_frames[f];
                const uint32_t o = s - sh.cell_begin[f];
                if (o < fr.capacity) {
                    emit_cell(fr, o, nrep, Cr, pr, ex, c3, ids, end - start);
                    if (fr.moff) glob(fr.moff)[o] = start - sh.key_begin[f];
                    if (fr.keys) {
                        uint64_t key;
                        if (no_sa) {
                            key = ids[0] - fr.pix_begin;
                        } else {
                            const CellCoord cc = coarse_cell(s_grids[f], pr[0]);
                            const int L = C.level[(uint64_t)f * G3 + cc.lin];
                            int loc[3];
                            fine_local(cc, L, loc);
                            key = canonical_key(cc, loc, P.Lmax);
                        }
                        glob(fr.keys)[o] = key;
                    }
                }
                atomicAdd(&sh.rcount[f], (uint32_t)nrep);
            }
        }
        wave_sync();
    }
    __syncthreads();
    for (uint32_t f = threadIdx.x; f < nf; f += kBlock)
        if (sh.rcount[f]) atomicAdd(&C.fs[f].R[item % kRSlots], sh.rcount[f]);
}

// ---------------------------------------------------------------- phase: final counts

__device__ __forceinline__ void ph_final(const Ctx& C, uint32_t, char*) {
    const CallHdr& H = *C.hdr;
    const bool no_sa = H.prm.flags & 4u;
    const uint32_t nf = H.n_frames;
    for (uint32_t f = threadIdx.x; f < nf; f += kBlock) {
        const DevFrame& fr = C.frames[f];
        const FrameState& st = C.fs[f];
        uint32_t S = 0;
        if (no_sa) {
            S = st.M;
        } else if (st.has_cells) {
            uint32_t next = C.bs->S_tot;
            for (uint32_t g = f + 1; g < nf; ++g)
                if (C.fs[g].has_cells) { next = C.fs[g].cell_begin; break; }
            S = next - st.cell_begin;
        }
        uint32_t R = 0;
        for (int k = 0; k < kRSlots; ++k) R += st.R[k];
        if (fr.moff && S <= fr.capacity) fr.moff[S] = st.M;
        *fr.count = S;
        *fr.status = (S > fr.capacity || (fr.mids && st.M > fr.member_capacity))
                         ? 1 : (C.bs->error ? 2 : 0);
        if (fr.info) {
            fr.info[0] = st.M;
            fr.info[1] = S;
            fr.info[2] = R;
            fr.info[3] = C.bs->key_bits;
        }
    }
}

}  // namespace ff
