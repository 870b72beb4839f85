// Structures shared by the host library and the gfx950 kernels of the fusion path.
#pragma once
#include <stdint.h>

namespace ff {

constexpr int kBlock = 256;              // threads per workgroup in every phase
constexpr int kWave = 64;                // CDNA wavefront
constexpr int kPxPerThread = 16;         // pixels per thread in the per-pixel phases
constexpr int kPxTile = kBlock * kPxPerThread;   // 4096 pixels per tile (never spans cameras)
constexpr int kScanTile = kBlock * 4;    // coarse cells per scan tile (256 workgroups for a 64^3 grid)
constexpr int kMaxPass = 16;             // radix passes
constexpr int kMaxRadixBits = 10;        // widest radix digit
constexpr int kMaxDigits = 1 << kMaxRadixBits;
constexpr int kMaxK = 8;                 // view budget K (own camera included)
constexpr int kMaxCamsPerFrame = 64;
constexpr int kMaxBatchCams = 1024;
constexpr int kMaxFrames = 64;
constexpr int kRSlots = 16;              // spread counters for representatives per frame
constexpr int kHashSlots = 2048;         // LDS hash of the coarse histogram
constexpr int kCountStripes = 4;         // copies of the coarse counts the histogram adds into
constexpr int kLdsCams = 256;            // cameras staged in LDS by the per-cell phase
constexpr int kEMin = -24, kEMax = 100;  // clamp of the coarse exponent
constexpr uint32_t kPad = 0xFFFFFFFFu;

// status bits the kernels raise in BatchState::error
constexpr uint32_t kErrBounds = 2u;      // an index failed a defensive bounds check

struct DevParams {
    float tau;
    int32_t K;
    float sigma;
    int32_t G, log2G, Lmax, target, level_override;
    uint32_t flags;
    uint32_t pad[3];
};

struct DevCam {
    float R[9];               // world -> camera rotation, row-major
    float t[3];
    float c[3];               // camera centre -R^T t (filled on the device)
    float fx, fy, cx, cy;
    int32_t W, H;
    uint32_t pix_off;         // first batch pixel id of this camera
    uint32_t frame_pix_off;   // first frame pixel id of this camera
    uint32_t tile_off;        // first pixel tile of this camera (batch numbering)
    uint32_t frame;           // frame index in the batch
    uint32_t rank;            // rank in its frame under (centre x, y, z, index) (device)
    uint32_t vec_ok;          // depth and conf 16-byte aligned
    uint32_t tab_off;         // first entry of this camera's ray tables (x then y)
    uint32_t pad0;
    const float* depth;
    const float* conf;
    const uint8_t* rgb;
    float* conf_out;          // Eq. 3 confidence written here before use (or null)
};

// the camera fields the per-cell phase needs, staged in LDS there
struct CamLite {
    float R[9];
    float t[3];
    float c[3];
    float fx, fy, cx, cy;
    int32_t W, H;
    uint32_t rank, pix_off;
    uint32_t frame;          // frame index in the batch
    uint32_t frame_cam;      // index of the camera within its frame (class mask bit)
    uint32_t tab_off;        // this camera's ray table: W column rays, then H row rays
    float invW;              // 1 / W, for a quick first guess of y = pixel / W
    // field-of-view fast path: cx + 1/2, cy + 1/2, and the largest floats below
    // W - m, H - m (clearly inside) and W + m, H + m (not clearly outside), m = 1/16 px
    float cxh, cyh, in_hx, in_hy, out_hx, out_hy;
    const float* depth;
    const float* conf;
    const uint8_t* rgb;
};

struct DevFrame {
    uint32_t cam_begin, n_cams;
    uint32_t pix_begin, n_pix;
    uint32_t tile_begin, n_tiles;
    uint32_t has_rgb, pad0;
    float* xyz;
    float* weight;
    uint8_t* rgb;
    uint32_t* n_members;
    uint32_t* reps;
    uint64_t* keys;
    uint32_t* moff;
    uint32_t* mids;
    uint32_t capacity, member_capacity;
    uint32_t* count;
    int32_t* status;
    uint32_t* info;
};

// Everything a call uploads: header, frames, cameras (device copy of a host staging slot).
struct CallHdr {
    DevParams prm;
    uint32_t n_frames, n_cams;
    uint32_t n_px_tiles, P_tot;
    uint32_t n_scan_tiles, n_sort_tiles;
    uint32_t n_cell_items, max_radix_bits;
    uint32_t npass_max, n_counts;
    uint32_t sort_items, lds_cams;
    uint32_t any_mids;
    uint32_t key64_ok;               // the key-width bound allows keys wider than 32 bits
    uint32_t cls_lanes;              // log2 of the camera slots per coarse cell (class phase)
    uint32_t hist_tiles;             // pixel tiles per coarse-histogram workgroup
};

// Field-of-view class of every camera of a frame for one occupied coarse cell: bit j of
// in_all is set when every point of the cell's box is in view of the frame's camera j by
// the exact float32 test, bit j of partial when neither that nor "no point is" could be
// shown (those points take the exact per-point test); cameras in neither mask see none.
struct CamClass {
    uint64_t in_all, partial;
};

// per pixel tile: AABB partial (order-preserving encodings) and gated count
struct TilePart {
    uint32_t mn[3], mx[3];
    uint32_t cnt, pad;
};

struct FrameState {
    uint32_t bmin_o[3], bmax_o[3];   // AABB (order-preserving encodings)
    float bmin[3];                   // AABB minimum
    float scale;                     // 2^-e, e the coarse exponent
    int32_t e;
    uint32_t M;                      // gated points
    uint32_t key_begin;              // first compacted/sorted position of the frame
    uint32_t cell_begin;             // first global cell of the frame
    uint32_t has_cells;
    uint32_t pad[3];
    uint64_t fine_begin;             // first dense fine index of the frame
    uint32_t R[kRSlots];             // representatives (spread counters, summed at the end)
};

struct BatchState {
    uint32_t M_tot, S_tot, error, key64;
    uint32_t key_bits, npass, pad0, pad1;
    uint64_t T_tot;
    uint32_t pass_shift[kMaxPass];
    uint32_t pass_bits[kMaxPass];
};

enum PhaseKind : uint32_t {
    PH_BACKPROJECT = 0, PH_TILE_REDUCE = 1, PH_HIST = 2, PH_SCAN_A = 3, PH_SCAN_M = 4,
    PH_SCAN_B = 5, PH_KEYS = 6, PH_RADIX_UP = 7, PH_RADIX_SCAN = 8, PH_RADIX_DOWN = 9,
    PH_HEAD_COUNT = 10, PH_HEAD_SCAN = 11, PH_HEAD_WRITE = 12, PH_CELLS = 13, PH_FINAL = 14,
    PH_CAM_PREP = 15, PH_CONF = 16, PH_CLASS = 17, PH_COUNT = 18
};

constexpr int kEmcBlocks = 2048;         // workgroups of the E_MC evaluator
constexpr int kMaxHistTiles = 8;         // pixel tiles per coarse-histogram workgroup (tuned)

// trace slots of the Eq. 3 confidence phase and of the camera classes (the radix passes
// use 16 .. 30; slots 7 .. 9 are not used by the radix kinds, which map to 16 ..)
constexpr int kTraceSlotConf = 31;
constexpr int kTraceSlotClass = 7;

// weights of Eq. 3
struct ConfWeights {
    float a, b, g, d;
};

}  // namespace ff
