// Internal types shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ssvb.h"

namespace ssvb {

constexpr int kLutSize = 4096;        // slice directions quantised to pi / 4096
constexpr int kLutOne = 4096;         // fixed-point 1.0 of the direction table
constexpr int kLatticeCapPx = 16383;  // hard cap on the projected radius, pixels
constexpr int kMaxDim = 16384;        // widest / tallest image the int32 lattice allows
constexpr int kMaxSlices = 64;
constexpr int kMaxSteps = 1024;

// Everything one frame's kernels need, by value in the kernel arguments.  Camera and
// sampling constants are derived on the host in FP64 and rounded once to FP32.
struct FrameArgs {
    // inputs
    const float* depth;
    const char* normal;
    const char* radiance;
    int64_t depth_pitch, normal_pitch, radiance_pitch;  // bytes
    int32_t normal_ch, radiance_ch;                     // 3 or 4
    int32_t normal_f16, radiance_f16;                   // element type flags
    // outputs
    float* ao;
    float* gi;
    float* amb;
    uint32_t* masks;
    int64_t ao_pitch, gi_pitch, amb_pitch, masks_pitch;  // bytes
    // image and camera
    int32_t W, H;
    float fx, fy, cx, cy;
    float inv_fx, inv_fy;   // 1 / fx, 1 / fy
    float d3x, d3y;         // 1 / (4096 fx), -1 / (4096 fy): view direction of one LUT unit
    float Rvw[9];           // view -> world rotation (ambient probe)
    // sampling
    int32_t nd, ns, na;
    int32_t nb;             // sectors: 32 or 128
    int32_t criterion, noise;
    int32_t step_dist;      // ssvb_step_distribution
    uint32_t ns_recip;      // floor(2^32 / (N_s + 1)), for quadratic steps
    uint32_t seed;
    uint32_t r2a1, r2a2, r2a3;
    float c_step;           // 16 radius fy / (N_s + 1), FP32
    float q_max_f;          // q_max as float (exact)
    int32_t q_min, q_max;   // step length bounds, 1/16 px
    float t0, tk;           // thickness t = t0 + tk * z
    float sh[27];           // ambient probe, [9][3]
    float amb_cb[32];       // cos of the subregion centre offsets -pi/2 + (k + 1/2) pi / N_a
    float amb_sb[32];       // sin of the same
    // slice-direction table (device), (Dx, Dy) pairs
    const int2* lut;
    // cos and sin of h pi / (2 N_b) for h = -2 N_b .. 2 N_b (device, FP64), index h + 2 N_b
    const double2* half_sector;
    // launch shape: tile_w x tile_h pixels per workgroup; tiles are walked in vertical
    // strips of `strip` tiles, and the walk is cut into one contiguous run per XCD
    int32_t tile_w, tile_h, tiles_x, tiles_y, strip;
    // pixels the gather computes: every pixel (sub = 1), or those with both coordinates
    // even (sub = 2, half resolution; the upsampler fills the rest)
    int32_t sub;
    // lanes per pixel: the N_d slices of a pixel are split over lp adjacent lanes;
    // tile_w * tile_h * lp = 256 threads per workgroup
    int32_t lp;
};

constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, each with its own L2

// A launch shape: tile of tile_w x tile_h pixels, strip width in tiles, lanes per pixel.
struct LaunchShape {
    int32_t tile_w, tile_h, strip, lp;
};
void set_launch(FrameArgs& A, LaunchShape L);

// Position `ord` of the strip walk over the frame's tiles -> tile (tx, ty).
__device__ __forceinline__ void walk_tile(const FrameArgs& A, uint32_t ord, int& tx, int& ty) {
    const uint32_t S = (uint32_t)A.strip, TY = (uint32_t)A.tiles_y;
    const uint32_t full = (uint32_t)A.tiles_x / S;
    if (ord < full * S * TY) {
        const uint32_t st = ord / (S * TY), r = ord % (S * TY);
        ty = (int)(r / S);
        tx = (int)(st * S + r % S);
    } else {
        const uint32_t wl = (uint32_t)A.tiles_x - full * S, r = ord - full * S * TY;
        ty = (int)(r / wl);
        tx = (int)(full * S + r % wl);
    }
}

// ---------------------------------------------------------------------------------------
// batched persistent path
// ---------------------------------------------------------------------------------------
constexpr int kMaxBatch = 64;  // frames per descriptor table (larger batches are chunked)
// queue heads: one per mask width and XCD
constexpr int kBatchQueues = 2 * kXcds;
// frames of at most this many tiles go into batches; larger ones get single-frame launches
// (a 1920x1080 frame in 32x8 tiles has 8,100)
constexpr uint32_t kPackTiles = 8192;
// kinds of frame in a batch; each set of kinds has its own captured graph
constexpr int kBatch32 = 1, kBatch128 = 2, kBatchHalf = 4, kBatchKinds = 8;

// Frames of one persistent launch.  For each mask width w (0: 32 sectors, 1: 128) the tile
// walks of that width's frames are laid end to end (frame plist[w][j] holds tiles
// prefix[w][j] .. prefix[w][j + 1] - 1) and the list is cut into kXcds runs of equal
// sample cost, run k (tiles split[w][k] .. split[w][k + 1] - 1) in queue w * kXcds + k.
struct BatchDesc {
    int32_t n_frames;
    int32_t pn[2];
    int32_t plist[2][kMaxBatch];
    uint32_t prefix[2][kMaxBatch + 1];
    uint32_t split[2][kXcds + 1];
    FrameArgs frames[kMaxBatch];
};

}  // namespace ssvb
