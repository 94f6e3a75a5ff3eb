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

// Slice-major order: the work items are (tile, slice) pairs, taken slice by slice over
// chunks of tiles of each XCD's run, so that the samples in flight on a die point into one
// wedge of directions; an item writes its slice's sums (kPartialFloats floats: AO, GI rgb,
// ambient rgb, unused) to a partial buffer at [slice][computed row][computed column] (one
// plane per slice, so a wave's records are contiguous), and a second pass adds the slices
// in order.
constexpr int kPartialFloats = 8;
typedef float PartialQuad __attribute__((ext_vector_type(4)));  // half a record: one 16-byte access

constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, each with its own L2

// A launch shape: tile of tile_w x tile_h pixels, strip width in tiles, lanes per pixel.
struct LaunchShape {
    int32_t tile_w, tile_h, strip, lp;
};
void set_launch(FrameArgs& A, LaunchShape L);

// ---------------------------------------------------------------------------------------
// index path of the gather kernels, from a work item to every byte offset they access.
// Host and device: the kernels call these, and a host build of them checks on the CPU
// that every access stays inside the frame's buffers.
// ---------------------------------------------------------------------------------------
#define SSVB_HD __host__ __device__ __forceinline__

// Run of walk positions [first, first + count) queued for XCD k: the walk over nt tiles cut
// into kXcds runs of ceil(nt / kXcds) (the last ones shorter or empty).
SSVB_HD void xcd_run(uint32_t nt, int k, uint32_t& first, uint32_t& count) {
    const uint32_t per = (nt + kXcds - 1) / kXcds;
    first = (uint32_t)k * per;
    count = first < nt ? min(per, nt - first) : 0u;
}

// Position `ord` of the strip walk over the frame's tiles -> tile (tx, ty).
SSVB_HD void walk_tile(const FrameArgs& A, uint32_t ord, int& tx, int& ty) {
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

// Pixel (x, y) of thread `thread` of a workgroup working on tile (tx, ty), and the thread's
// lane `li` among the lp lanes that share the pixel.  The caller skips pixels with
// x >= W or y >= H (the frame's last tile row and column may be partial).
SSVB_HD void tile_pixel(const FrameArgs& A, int tx, int ty, int thread, int& x, int& y, int& li) {
    const int lp = A.lp, px = thread / lp;
    li = thread & (lp - 1);
    x = (tx * A.tile_w + px % A.tile_w) * A.sub;
    y = (ty * A.tile_h + px / A.tile_w) * A.sub;
}

// Offset of step j (0-based) from the pixel centre along the slice, in 1/16 pixel.
// Uniform steps (Algorithm 1): (j + 1 + xi) steps of q, jit = (q xi8) >> 8.  Quadratic
// steps (Section 4.3: denser near the pixel): the reach q (N_s + 1) times
// ((j + 1 + xi) / (N_s + 1))^2, in integers: ((q a^2) >> 16) * floor(2^32 / (N_s + 1))
// >> 32 with a = 256 (j + 1) + xi8 (q a^2 < 2^44, the second product < 2^50).
template <bool QUAD>
SSVB_HD int step_offset(const FrameArgs& A, int q, int jit, int xi8, int j) {
    if (!QUAD) return q * (j + 1) + jit;
    const uint64_t a = (uint64_t)(uint32_t)((j + 1) * 256 + xi8);
    const uint64_t t = ((uint64_t)(uint32_t)q * (a * a)) >> 16;
    return (int)((t * (uint64_t)A.ns_recip) >> 32);
}

// Lattice coordinate of a sample: c16 = (pixel << 16) + 2^15 (the pixel centre in 1/65536
// px), so = the signed step offset in 1/16 px, d = the direction component in 1/4096;
// arithmetic shift = floor.  |c16 + so d| < 2^31 for frames of at most kMaxDim pixels and
// offsets below kLatticeCapPx pixels.
SSVB_HD int lattice_coord(int c16, int so, int d) { return (c16 + so * d) >> 16; }

// Byte offsets in the images (every image spans less than 4 GiB: 32-bit offsets).
SSVB_HD uint32_t depth_off(const FrameArgs& A, int X, int Y) {
    return (uint32_t)Y * (uint32_t)A.depth_pitch + (uint32_t)X * 4u;
}
SSVB_HD uint32_t image_off(int64_t pitch, int ch, bool f16, int x, int y) {
    return (uint32_t)y * (uint32_t)pitch + (uint32_t)(x * ch) * (f16 ? 2u : 4u);
}
// Slice-major order: item j of a run of `count` tiles (count * nd items) is slice `slice` of
// the run's tile `tile`.  The run is cut into chunks of `chunk` tiles (the last may be
// shorter); a chunk's items are its tiles for slice 0, then for slice 1, and so on.
SSVB_HD void slice_item(uint32_t chunk, int nd, uint32_t count, uint32_t j, uint32_t& tile, int& slice) {
    const uint32_t per = chunk * (uint32_t)nd;  // items of a full chunk
    const uint32_t c = j / per, r = j - c * per;
    const uint32_t first = c * chunk;
    const uint32_t n = min(chunk, count - first);  // tiles of this chunk
    slice = (int)(r / n);
    tile = first + r % n;
}

// Offset (floats) of the partial sums of slice s of the computed pixel (x, y).
SSVB_HD int64_t partial_off(const FrameArgs& A, int x, int y, int s) {
    const int64_t gw = (A.W + A.sub - 1) / A.sub, gh = (A.H + A.sub - 1) / A.sub;
    return (((int64_t)s * gh + y / A.sub) * gw + x / A.sub) * kPartialFloats;
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

// Frame (index into plist[w]) of tile g of width w's list.  `j` is the caller's cursor: the
// frame of its previous tile (0 at first); runs are claimed in increasing order, so the
// search usually moves forward by a few frames.  Requires g < prefix[w][pn[w]].
SSVB_HD int batch_frame(const BatchDesc& D, int w, uint32_t g, int j) {
    if (g < D.prefix[w][j]) j = 0;
    while (D.prefix[w][j + 1] <= g) ++j;
    return j;
}

}  // namespace ssvb
