// Structures shared by the host library and the gfx950 kernels of the fusion path.
#pragma once
#include <stdint.h>

namespace ff {

constexpr int kBlock = 256;              // threads per workgroup in every phase
constexpr int kWave = 64;                // CDNA wavefront
constexpr int kPxPerThread = 16;         // pixels per thread in the per-pixel phases
constexpr int kPxTile = kBlock * kPxPerThread;   // 4096 pixels per tile (never spans cameras)
constexpr int kScanTile = kBlock * 16;   // coarse cells per scan tile
constexpr int kMaxPass = 16;             // radix passes (4-bit digits over 64-bit keys)
constexpr int kMaxDigits = 256;          // 8-bit digits at most
constexpr int kMaxK = 8;                 // view budget K (own camera included)
constexpr int kMaxCamsPerFrame = 64;
constexpr int kMaxBatchCams = 1024;
constexpr int kMaxFrames = 64;
constexpr int kMaxPhases = 40;
constexpr int kEMin = -24, kEMax = 100;  // clamp of the coarse exponent
constexpr uint32_t kPad = 0xFFFFFFFFu;

// status bits the kernels raise in BatchState::error
constexpr uint32_t kErrSpin = 1u;        // a bounded wait gave up (never expected)
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
    uint32_t n_cell_items, radix_bits;
    uint32_t npass_max, n_phases;
    uint64_t wait_ticks;                    // wall-clock bound of any single wait
    uint32_t phase_begin[kMaxPhases + 1];   // persistent schedule: first ticket of each phase
    uint32_t phase_kind[kMaxPhases];
};

struct FrameState {
    uint32_t bmin_o[3], bmax_o[3];   // order-preserving encodings of the AABB
    uint32_t M, S, R, pad;
    uint64_t fine_begin;             // first dense fine index of the frame
};

struct BatchState {
    uint32_t tickets[kMaxPhases];
    uint32_t done[kMaxPhases];
    uint32_t M_tot, S_tot, error, key64;
    uint32_t key_bits, npass, pad0, pad1;
    uint64_t T_tot;
    uint32_t digit_hist[kMaxPass][kMaxDigits];
};

enum PhaseKind : uint32_t {
    PH_BACKPROJECT = 0, PH_HIST = 1, PH_SCAN_A = 2, PH_SCAN_M = 3, PH_SCAN_B = 4,
    PH_KEYS = 5, PH_HEADS = 6, PH_CELLS = 7, PH_FINAL = 8,
    PH_RADIX = 16      // + pass index
};

}  // namespace ff
