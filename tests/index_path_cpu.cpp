// Host emulation of the gather kernels' index path, for the CPU test suite.
//
// The kernels' index functions (XCD runs, tile walk, tile -> pixel, batch cursor, step
// offsets, lattice, image offsets) are __host__ __device__ and are called here as written;
// the frame constants come from the library's own fill_frame / build_batch (its sources
// are built into the test program, their host code under the sanitizers too; no GPU
// needed).  For every frame and launch shape below the emulation claims every work
// item the way the persistent kernels do and checks, with bounds assertions (and ASan /
// UBSan in the test build), that
//   - every tile of every frame is claimed exactly once, and every computed pixel is
//     reached by exactly lp lanes (each lane once) and lies inside the frame;
//   - every byte the pixel's code reads (own depth, normal, radiance) or writes (AO, GI,
//     ambient, slice masks) lies inside its buffer, and every input offset the kernels
//     form in 32 bits, for any texel a sample can land on, equals the exact one;
//   - the integer lattice never overflows int32 at the frame's extreme pixels, longest
//     offsets and every direction of the slice-direction table;
//   - sampled texels pass the kernels' on-screen test only inside the frame;
//   - in slice-major order, every (tile, slice) item is produced once, every computed
//     pixel's every slice record lands once at its exact offset inside the partial
//     buffer, and the reduction reads each pixel's records once, inside the buffer.
// The half-resolution fill (upsample_pixel) and every denoiser pass (stage_cell and
// filter_cell over LDS-sized arrays) also run on real host buffers of exactly the bytes
// the frame's pitches span, so the sanitizer reports any access outside them.
// It runs the library's strip walk and, with --interleaved, a reconstruction of the
// interleaved strip walk (strips 0, 8, 16, ... then 1, 9, 17, ...) that was timed and then
// withdrawn.  With --fuzz N SEED it draws N random inputs instead (see fuzz() below); with
// --part k/n it runs every n-th frame shape from the k-th (the batches in the last part).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "ssvb_denoise_cell.h"
#include "ssvb_host.h"
#include "ssvb_pixel.h"

using namespace ssvb;

static long g_checks = 0, g_fail = 0;

#define CHECK(cond, ...)                                                     \
    do {                                                                     \
        ++g_checks;                                                          \
        if (!(cond)) {                                                       \
            if (++g_fail <= 20) {                                            \
                printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond);       \
                printf(__VA_ARGS__);                                         \
                printf("\n");                                                \
            }                                                                \
        }                                                                    \
    } while (0)

// ---------------------------------------------------------------------------------------
// the withdrawn interleaved walk, reconstructed: strips (S tiles wide, the last one
// possibly narrower) are visited in the order 0, 8, 16, ..., 1, 9, 17, ..., 7, 15, ...
// ---------------------------------------------------------------------------------------
static void walk_interleaved(const FrameArgs& A, uint32_t ord, int& tx, int& ty) {
    const uint32_t S = (uint32_t)A.strip, TY = (uint32_t)A.tiles_y, TX = (uint32_t)A.tiles_x;
    const uint32_t nstrips = (TX + S - 1) / S, full = TX / S, wl = TX - full * S;
    uint32_t base = 0;
    for (uint32_t g = 0; g < (uint32_t)kXcds && g < nstrips; ++g) {
        const uint32_t in_group = (nstrips - g + kXcds - 1) / kXcds;  // strips g, g + 8, ...
        uint32_t tiles = in_group * S * TY;
        const bool has_partial = wl != 0 && (nstrips - 1) % kXcds == g;
        if (has_partial) tiles -= (S - wl) * TY;
        if (ord < base + tiles) {
            const uint32_t r = ord - base, st_local = r / (S * TY), rr = r % (S * TY);
            const uint32_t strip = g + (uint32_t)kXcds * st_local;
            const uint32_t width = (wl != 0 && strip == nstrips - 1) ? wl : S;
            ty = (int)(rr / width);
            tx = (int)(strip * S + rr % width);
            return;
        }
        base += tiles;
    }
    tx = ty = -1;  // past the end: reported by the caller
}

static bool g_interleaved = false;

static void walk(const FrameArgs& A, uint32_t ord, int& tx, int& ty) {
    if (g_interleaved) walk_interleaved(A, ord, tx, ty);
    else walk_tile(A, ord, tx, ty);
}

// ---------------------------------------------------------------------------------------
// buffers of one frame (byte sizes only: nothing is allocated)
// ---------------------------------------------------------------------------------------
struct Frame {
    int W, H, nd, ns, nb, sub, dist, min_q4;
    bool n16, r16;
    int nch, rch;
    int pad;  // extra bytes per row in every pitch
    bool masks;
    float radius;
};

struct Sizes {
    int64_t depth, normal, radiance, ao, gi, amb, masks;
};

static int64_t span(int64_t pitch, int H, int64_t row) { return pitch * (H - 1) + row; }

static Sizes sizes_of(const FrameArgs& A) {
    Sizes s;
    const int W = A.W, H = A.H;
    s.depth = span(A.depth_pitch, H, (int64_t)W * 4);
    s.normal = span(A.normal_pitch, H, (int64_t)W * A.normal_ch * (A.normal_f16 ? 2 : 4));
    s.radiance = span(A.radiance_pitch, H, (int64_t)W * A.radiance_ch * (A.radiance_f16 ? 2 : 4));
    s.ao = span(A.ao_pitch, H, (int64_t)W * 4);
    s.gi = span(A.gi_pitch, H, (int64_t)W * 12);
    s.amb = span(A.amb_pitch, H, (int64_t)W * 12);
    s.masks = A.masks ? span(A.masks_pitch, H, (int64_t)W * A.nd * (A.nb / 32) * 4) : 0;
    return s;
}

// The library's frame constants for a frame description (fake, distinct base addresses:
// only offsets are checked).
static void make_frame(const Frame& f, LaunchShape shape, bool forced, FrameArgs& A, ssvb_frame* out_frame = nullptr) {
    static FrameTables tab;
    tab.forced = forced;
    tab.force = shape;
    ssvb_camera cam{f.W, f.H, 0.5f * f.H, 0.5f * f.H, 0.5f * f.W, 0.5f * f.H, {1, 0, 0, 0, 1, 0, 0, 0, 1}};
    ssvb_params p;
    ssvb_default_params(&p);
    p.slices = f.nd;
    p.steps = f.ns;
    p.sectors = f.nb;
    p.radius = f.radius;
    p.resolution = f.sub;
    p.step_distribution = f.dist;
    p.min_step_q4 = f.min_q4;
    const int ne = f.n16 ? 2 : 4, re = f.r16 ? 2 : 4;
    ssvb_image depth{(const void*)0x10000000, f.pad ? (int64_t)f.W * 4 + f.pad * 4 : 0, SSVB_F32, 1};
    ssvb_image normal{(const void*)0x20000000, f.pad ? (int64_t)f.W * f.nch * ne + f.pad * ne : 0,
                      f.n16 ? SSVB_F16 : SSVB_F32, f.nch};
    ssvb_image radiance{(const void*)0x30000000, f.pad ? (int64_t)f.W * f.rch * re + f.pad * re : 0,
                        f.r16 ? SSVB_F16 : SSVB_F32, f.rch};
    ssvb_outputs o{(float*)0x40000000, (float*)0x50000000, (float*)0x60000000,
                   f.masks ? (uint32_t*)0x70000000 : nullptr,
                   f.pad ? (int64_t)f.W * 4 + f.pad * 4 : 0, f.pad ? (int64_t)f.W * 12 + f.pad * 4 : 0,
                   f.pad ? (int64_t)f.W * 12 + f.pad * 4 : 0,
                   f.pad ? (int64_t)f.W * f.nd * (f.nb / 32) * 4 + f.pad * 4 : 0};
    CHECK(ssvb_validate(&depth, &normal, &radiance, &cam, &p, &o) == SSVB_OK, "frame %dx%d rejected: %s", f.W, f.H,
          ssvb_last_error());
    fill_frame(A, &tab, &depth, &normal, &radiance, &cam, &p, &o);
    if (out_frame) *out_frame = ssvb_frame{depth, normal, radiance, cam, p, o};
}

// Everything one pixel's code touches, as the kernels compute it.
static void check_pixel(const FrameArgs& A, const Sizes& S, int x, int y, int li) {
    CHECK(x >= 0 && x < A.W && y >= 0 && y < A.H, "pixel (%d, %d) outside %dx%d", x, y, A.W, A.H);
    CHECK(x % A.sub == 0 && y % A.sub == 0, "pixel (%d, %d) not on the computed grid (sub %d)", x, y, A.sub);
    CHECK(li >= 0 && li < A.lp, "lane %d of %d", li, A.lp);
    // the kernels' 32-bit offsets equal the exact ones (no wrap can land inside the buffer
    // at the wrong texel) and lie inside the buffer
    const int64_t d = depth_off(A, x, y);
    CHECK(d == (int64_t)y * A.depth_pitch + 4 * (int64_t)x, "depth offset %lld wrapped", (long long)d);
    CHECK(d >= 0 && d + 4 <= S.depth, "depth offset %lld of %lld", (long long)d, (long long)S.depth);
    const int64_t n = image_off(A.normal_pitch, A.normal_ch, A.normal_f16, x, y);
    CHECK(n == (int64_t)y * A.normal_pitch + (int64_t)x * A.normal_ch * (A.normal_f16 ? 2 : 4),
          "normal offset %lld wrapped", (long long)n);
    CHECK(n + 3 * (A.normal_f16 ? 2 : 4) <= S.normal, "normal offset %lld of %lld", (long long)n, (long long)S.normal);
    const int64_t r = image_off(A.radiance_pitch, A.radiance_ch, A.radiance_f16, x, y);
    CHECK(r == (int64_t)y * A.radiance_pitch + (int64_t)x * A.radiance_ch * (A.radiance_f16 ? 2 : 4),
          "radiance offset %lld wrapped", (long long)r);
    CHECK(r + 3 * (A.radiance_f16 ? 2 : 4) <= S.radiance, "radiance offset %lld", (long long)r);
    // outputs, as the kernels address them (row pointer + element)
    CHECK((int64_t)y * A.ao_pitch + (int64_t)x * 4 + 4 <= S.ao, "ao (%d, %d)", x, y);
    CHECK((int64_t)y * A.gi_pitch + 12 * (int64_t)x + 12 <= S.gi, "gi (%d, %d)", x, y);
    CHECK((int64_t)y * A.amb_pitch + 12 * (int64_t)x + 12 <= S.amb, "ambient (%d, %d)", x, y);
    if (A.masks) {
        const int words = A.nb / 32;
        for (int i = li; i < A.nd; i += A.lp) {
            const int64_t m = (int64_t)y * A.masks_pitch + 4 * ((int64_t)x * A.nd * words + (int64_t)i * words);
            CHECK(m >= 0 && m + 4 * words <= S.masks, "masks (%d, %d) slice %d", x, y, i);
        }
    }
}

// Every texel a sample can land on (any pixel of the frame, computed or not): the depth,
// normal and radiance offsets the kernels form for it are exact and inside the images.
static void check_texels(const FrameArgs& A, const Sizes& S) {
    const int ne = A.normal_f16 ? 2 : 4, re = A.radiance_f16 ? 2 : 4;
    for (int Y = 0; Y < A.H; ++Y)
        for (int X = 0; X < A.W; ++X) {
            const int64_t d = depth_off(A, X, Y), n = image_off(A.normal_pitch, A.normal_ch, A.normal_f16, X, Y),
                          r = image_off(A.radiance_pitch, A.radiance_ch, A.radiance_f16, X, Y);
            CHECK(d == (int64_t)Y * A.depth_pitch + 4 * (int64_t)X && d + 4 <= S.depth, "texel (%d, %d) depth", X, Y);
            CHECK(n == (int64_t)Y * A.normal_pitch + (int64_t)X * A.normal_ch * ne && n + 3 * ne <= S.normal,
                  "texel (%d, %d) normal", X, Y);
            CHECK(r == (int64_t)Y * A.radiance_pitch + (int64_t)X * A.radiance_ch * re && r + 3 * re <= S.radiance,
                  "texel (%d, %d) radiance", X, Y);
        }
}

// One frame as gather_frame runs it: 8 XCD runs of the walk, 256 threads per tile.
static void emulate_frame(const FrameArgs& A) {
    const Sizes S = sizes_of(A);
    const uint32_t nt = (uint32_t)A.tiles_x * (uint32_t)A.tiles_y;
    std::vector<uint8_t> tile_seen(nt, 0);
    std::vector<uint8_t> lanes((size_t)A.W * A.H, 0);
    uint32_t claimed = 0;
    for (int k = 0; k < kXcds; ++k) {
        uint32_t first, count;
        xcd_run(nt, k, first, count);
        CHECK(count == 0 || first + count <= nt, "run %d: [%u, %u) of %u", k, first, first + count, nt);
        for (uint32_t item = 0; item < count; ++item) {
            int tx = -1, ty = -1;
            walk(A, first + item, tx, ty);
            ++claimed;
            CHECK(tx >= 0 && tx < A.tiles_x && ty >= 0 && ty < A.tiles_y, "walk %u -> tile (%d, %d) of %dx%d",
                  first + item, tx, ty, A.tiles_x, A.tiles_y);
            if (!(tx >= 0 && tx < A.tiles_x && ty >= 0 && ty < A.tiles_y)) continue;
            CHECK(tile_seen[(size_t)ty * A.tiles_x + tx]++ == 0, "tile (%d, %d) claimed twice", tx, ty);
            for (int t = 0; t < 256; ++t) {
                int x, y, li;
                tile_pixel(A, tx, ty, t, x, y, li);
                if (x < A.W && y < A.H) {  // the kernels' guard
                    check_pixel(A, S, x, y, li);
                    if (x >= 0 && y >= 0) lanes[(size_t)y * A.W + x]++;
                }
            }
        }
    }
    CHECK(claimed == nt, "%u of %u tiles claimed", claimed, nt);
    long wrong = 0;
    for (int y = 0; y < A.H; ++y)
        for (int x = 0; x < A.W; ++x) {
            const int want = (x % A.sub == 0 && y % A.sub == 0) ? A.lp : 0;
            wrong += lanes[(size_t)y * A.W + x] != want;
        }
    CHECK(wrong == 0, "%ld pixels not reached by exactly lp lanes (%dx%d, tile %dx%d, strip %d, lp %d, sub %d)", wrong,
          A.W, A.H, A.tile_w, A.tile_h, A.strip, A.lp, A.sub);
    check_texels(A, S);
}

// One frame in slice-major order as the library launches it (lanes per pixel forced to 1,
// then gather_slices and reduce_slices): every (tile, slice) item of every XCD run is
// produced exactly once by slice_item, every computed pixel's every slice is written once
// at its exact offset inside the partial buffer, the slice's mask words lie inside the mask
// image, and the reduction's grid reads each computed pixel's partial sums once, inside
// the buffer, and writes its outputs inside the images.
static long g_slice_items = 0;
static void emulate_slices(const FrameArgs& A0, uint32_t chunk) {
    FrameArgs A = A0;
    if (A.lp > 1) set_launch(A, LaunchShape{A.tile_w * A.lp, A.tile_h, A.strip, 1});
    CHECK(A.lp == 1 && A.tile_w * A.tile_h == 256, "slice-major shape %dx%d lp %d", A.tile_w, A.tile_h, A.lp);
    const Sizes S = sizes_of(A);
    const int64_t gw = (A.W + A.sub - 1) / A.sub, gh = (A.H + A.sub - 1) / A.sub;
    const int64_t floats = gw * gh * A.nd * kPartialFloats;
    const int words = A.nb / 32;
    std::vector<uint8_t> seen((size_t)(gw * gh * A.nd), 0);
    const uint32_t nt = (uint32_t)A.tiles_x * (uint32_t)A.tiles_y;
    for (int k = 0; k < kXcds; ++k) {
        uint32_t first, count;
        xcd_run(nt, k, first, count);
        CHECK((uint64_t)count * (uint64_t)A.nd < ((uint64_t)1 << 32), "run of %u tiles x %d slices", count, A.nd);
        std::vector<uint8_t> item_seen((size_t)count * A.nd, 0);
        for (uint32_t j = 0; j < count * (uint32_t)A.nd; ++j) {
            uint32_t tile = ~0u;
            int slice = -1, tx = -1, ty = -1;
            slice_item(chunk, A.nd, count, j, tile, slice);
            ++g_slice_items;
            CHECK(tile < count && slice >= 0 && slice < A.nd, "item %u -> tile %u slice %d (run of %u, chunk %u)", j,
                  tile, slice, count, chunk);
            if (!(tile < count && slice >= 0 && slice < A.nd)) continue;
            CHECK(item_seen[(size_t)tile * A.nd + slice]++ == 0, "tile %u slice %d twice", tile, slice);
            walk_tile(A, first + tile, tx, ty);
            CHECK(tx >= 0 && tx < A.tiles_x && ty >= 0 && ty < A.tiles_y, "tile (%d, %d)", tx, ty);
            for (int t = 0; t < 256; ++t) {
                int x, y, li;
                tile_pixel(A, tx, ty, t, x, y, li);
                if (!(x < A.W && y < A.H)) continue;
                CHECK(x >= 0 && y >= 0 && x % A.sub == 0 && y % A.sub == 0 && li == 0, "pixel (%d, %d)", x, y);
                const int64_t off = partial_off(A, x, y, slice);
                const int64_t cell = ((int64_t)slice * gh + y / A.sub) * gw + x / A.sub;
                CHECK(off == cell * kPartialFloats && off >= 0 && off + kPartialFloats <= floats,
                      "partial offset %lld of %lld floats, pixel (%d, %d) slice %d", (long long)off, (long long)floats,
                      x, y, slice);
                if (off == cell * kPartialFloats && off >= 0 && off + kPartialFloats <= floats) seen[(size_t)cell]++;
                if (A.masks) {
                    const int64_t m =
                        (int64_t)y * A.masks_pitch + 4 * ((int64_t)x * A.nd * words + (int64_t)slice * words);
                    CHECK(m >= 0 && m + 4 * words <= S.masks, "masks (%d, %d) slice %d", x, y, slice);
                }
            }
        }
    }
    long wrong = 0;
    for (uint8_t c : seen) wrong += c != 1;
    CHECK(wrong == 0, "%ld (pixel, slice) partial records not written exactly once (%dx%d, %d slices, chunk %u)",
          wrong, A.W, A.H, A.nd, chunk);
    // reduce_slices: 16 x 16 blocks of the computed grid
    std::vector<uint8_t> red((size_t)(gw * gh), 0);
    const int bx = (int)((gw + 15) / 16), by = (int)((gh + 15) / 16);
    for (int b = 0; b < by; ++b)
        for (int a = 0; a < bx; ++a)
            for (int t = 0; t < 256; ++t) {
                const int u = a * 16 + t % 16, v = b * 16 + t / 16;
                if (!(u < gw && v < gh)) continue;
                const int x = u * A.sub, y = v * A.sub;
                for (int sl = 0; sl < A.nd; ++sl) {
                    const int64_t p0 = partial_off(A, x, y, sl);
                    CHECK(p0 >= 0 && p0 % 4 == 0 && p0 + kPartialFloats <= floats, "reduction of (%d, %d) slice %d", x,
                          y, sl);
                }
                check_pixel(A, S, x, y, 0);
                red[(size_t)v * gw + u]++;
            }
    wrong = 0;
    for (uint8_t c : red) wrong += c != 1;
    CHECK(wrong == 0, "%ld computed pixels not reduced exactly once", wrong);
}

// ---------------------------------------------------------------------------------------
// the half-resolution fill and the denoiser on real host buffers of exactly the bytes the
// frame's pitches span (AddressSanitizer reports any access outside them)
// ---------------------------------------------------------------------------------------
struct Span {
    std::vector<char> b;
    explicit Span(int64_t n) : b((size_t)n) {}
    char* p() { return b.data(); }
};

// A depth image with background pixels in it (every 7th and the border of some rows).
static void fill_depth(const FrameArgs& A, char* d) {
    for (int y = 0; y < A.H; ++y)
        for (int x = 0; x < A.W; ++x) {
            float z = 1.0f + (float)((x * 7 + y * 3) % 11);
            if ((x + 2 * y) % 7 == 0 || (y % 5 == 0 && x == 0)) z = 0.0f;
            memcpy(d + (int64_t)y * A.depth_pitch + 4 * (int64_t)x, &z, 4);
        }
}

// upsample_pixel on every pixel of a half-resolution frame (each thread's view of it).
static long check_upsample(const FrameArgs& A0) {
    const Sizes S = sizes_of(A0);
    Span depth(S.depth), ao(S.ao), gi(S.gi), amb(S.amb);
    FrameArgs A = A0;
    A.depth = (const float*)depth.p();
    A.ao = (float*)ao.p(), A.gi = (float*)gi.p(), A.amb = (float*)amb.p();
    fill_depth(A, depth.p());
    for (int y = 0; y < A.H; ++y)
        for (int x = 0; x < A.W; ++x) upsample_pixel(A, x, y);
    return (long)A.W * A.H;
}

// Every pass of the denoiser (taps 1, 2 and 4 cells apart; normal power 16 by squarings and
// 3 by square-and-multiply) on the frame's geometry and pitches, at its resolution: each
// 16 x 16-cell tile staged into LDS-sized arrays and filtered as a workgroup does.
template <int S, int K2>
static void denoise_tiles(const DenoiseArgs& D) {
    constexpr int E = kDenoiseTile + 4 * S, N = E * E;
    std::vector<float4> sA(N), sB(N), sC(N);  // exactly the kernel's LDS arrays
    for (int tile = 0; tile < D.tiles; ++tile) {
        const int u0 = (tile % D.tiles_x) * kDenoiseTile - 2 * S;
        const int v0 = (tile / D.tiles_x) * kDenoiseTile - 2 * S;
        for (int i = 0; i < N; ++i) {
            const int u = u0 + i % E, v = v0 + i / E;
            float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a, c = a;
            if (u >= 0 && v >= 0 && u < D.gw && v < D.gh) dn::stage_cell(D, u, v, a, b, c);
            sA[(size_t)i] = a;
            sB[(size_t)i] = b;
            sC[(size_t)i] = c;
        }
        for (int t = 0; t < kDenoiseTile * kDenoiseTile; ++t)
            dn::filter_cell<S, K2>(D, sA.data(), sB.data(), sC.data(), u0, v0, t % kDenoiseTile, t / kDenoiseTile);
    }
}

static long check_denoise(const FrameArgs& A0) {
    const Sizes S = sizes_of(A0);
    Span depth(S.depth), normal(S.normal), in_ao(S.ao), in_gi(S.gi), in_amb(S.amb), out_ao(S.ao), out_gi(S.gi),
        out_amb(S.amb);
    FrameArgs A = A0;
    A.depth = (const float*)depth.p();
    fill_depth(A, depth.p());
    memset(normal.p(), 0, normal.b.size());
    const ssvb_image d{depth.p(), A.depth_pitch, SSVB_F32, 1};
    const ssvb_image n{normal.p(), A.normal_pitch, A.normal_f16 ? SSVB_F16 : SSVB_F32, A.normal_ch};
    const ssvb_camera cam{A.W, A.H, 0.5f * A.H, 0.5f * A.H, 0.5f * A.W, 0.5f * A.H, {1, 0, 0, 0, 1, 0, 0, 0, 1}};
    const ssvb_outputs in{(float*)in_ao.p(), (float*)in_gi.p(), (float*)in_amb.p(), nullptr, A.ao_pitch, A.gi_pitch,
                          A.amb_pitch, 0};
    const ssvb_outputs out{(float*)out_ao.p(), (float*)out_gi.p(), (float*)out_amb.p(), nullptr, A.ao_pitch,
                           A.gi_pitch, A.amb_pitch, 0};
    memset(in_ao.p(), 0, in_ao.b.size());
    memset(in_gi.p(), 0, in_gi.b.size());
    memset(in_amb.p(), 0, in_amb.b.size());
    long cells = 0;
    for (int power : {16, 3}) {
        const ssvb_denoise_params dp{3, power, 0.05f, A.sub};
        DenoiseArgs D;
        fill_denoise(D, &d, &n, &cam, &dp, &in, &out);
        CHECK(D.gw == (A.W + A.sub - 1) / A.sub && D.gh == (A.H + A.sub - 1) / A.sub, "denoise grid %dx%d", D.gw, D.gh);
        if (power == 16) {
            denoise_tiles<1, 4>(D);
            denoise_tiles<2, 4>(D);
            denoise_tiles<4, 4>(D);
        } else {
            denoise_tiles<1, -1>(D);
            denoise_tiles<2, -1>(D);
            denoise_tiles<4, -1>(D);
        }
        cells += 3L * D.gw * D.gh;
    }
    return cells;
}

static long g_upsampled = 0, g_denoised = 0;

// The lattice at the frame's extreme pixels, for the longest offsets and every direction
// of the table (computed as the library builds it): no int32 overflow, and a texel that
// passes the on-screen test lies inside the frame.
static void check_lattice(const FrameArgs& A) {
    const int xs[2] = {0, ((A.W - 1) / A.sub) * A.sub}, ys[2] = {0, ((A.H - 1) / A.sub) * A.sub};
    const int qs[2] = {A.q_min, A.q_max};
    const int xis[2] = {0, 255};
    for (int k = 0; k < kLutSize; k += 1) {
        const double phi = M_PI * k / kLutSize;
        const int dx = (int)floor(kLutOne * cos(phi) + 0.5), dy = (int)floor(kLutOne * sin(phi) + 0.5);
        for (int q : qs)
            for (int xi8 : xis)
                for (int j : {0, A.ns - 1})
                    for (int s : {1, -1}) {
                        const int jit = (q * xi8) >> 8;
                        const int o = A.step_dist == SSVB_STEPS_QUADRATIC ? step_offset<true>(A, q, jit, xi8, j)
                                                                          : step_offset<false>(A, q, jit, xi8, j);
                        CHECK(o >= 0 && o < 16 * (kLatticeCapPx + 1), "offset %d (q %d, j %d)", o, q, j);
                        for (int x : xs)
                            for (int y : ys) {
                                const int64_t X64 = (((int64_t)x << 16) + 32768 + (int64_t)s * o * dx) >> 16;
                                const int64_t Y64 = (((int64_t)y << 16) + 32768 + (int64_t)s * o * dy) >> 16;
                                const int64_t sx = ((int64_t)x << 16) + 32768 + (int64_t)s * o * dx;
                                const int64_t sy = ((int64_t)y << 16) + 32768 + (int64_t)s * o * dy;
                                CHECK(sx >= INT32_MIN && sx <= INT32_MAX && sy >= INT32_MIN && sy <= INT32_MAX,
                                      "lattice overflow at (%d, %d), offset %d, direction %d", x, y, o, k);
                                const int X = lattice_coord((x << 16) + 32768, s * o, dx);
                                const int Y = lattice_coord((y << 16) + 32768, s * o, dy);
                                CHECK(X == X64 && Y == Y64, "lattice (%d, %d) != (%lld, %lld)", X, Y, (long long)X64,
                                      (long long)Y64);
                                if ((unsigned)X < (unsigned)A.W && (unsigned)Y < (unsigned)A.H) {
                                    const int64_t d = depth_off(A, X, Y);
                                    CHECK(d == (int64_t)Y * A.depth_pitch + 4 * (int64_t)X, "texel (%d, %d) wrapped", X, Y);
                                    CHECK(d + 4 <= sizes_of(A).depth, "texel (%d, %d)", X, Y);
                                }
                            }
                    }
    }
}

// A batch as gather_batch runs it: per mask width, 8 runs of the packed tile list, claimed
// by `wgs` workgroups in turn (each starting at its own XCD's run and keeping its frame
// cursor across claims, as the kernel does).
static void emulate_batch_frames(const std::vector<ssvb_frame>& F, const std::vector<FrameArgs>& A,
                                 const FrameTables& tab, int wgs) {
    static BatchDesc D;
    memset(&D, 0, sizeof D);
    // the descriptor as the library builds it for a context with this launch shape
    build_batch(&tab, &D, F.data(), (int)F.size());
    // the descriptor's frame constants are the single-frame launch's, byte for byte (both
    // come from fill_frame, which clears the padding), so a batched frame runs the same
    // per-pixel code on the same constants as its own launch
    CHECK(D.n_frames == (int)F.size(), "batch of %d frames, descriptor %d", (int)F.size(), D.n_frames);
    for (size_t i = 0; i < F.size(); ++i)
        CHECK(memcmp(&D.frames[i], &A[i], sizeof(FrameArgs)) == 0, "frame %zu: batch constants differ", i);
    for (int w = 0; w < 2; ++w) {
        const int pn = D.pn[w];
        const uint32_t total = pn ? D.prefix[w][pn] : 0;
        CHECK(D.split[w][0] == 0 && D.split[w][kXcds] == total, "width %d: runs [%u, %u) of %u tiles", w,
              D.split[w][0], D.split[w][kXcds], total);
        for (int k = 0; k < kXcds; ++k) CHECK(D.split[w][k] <= D.split[w][k + 1], "width %d run %d reversed", w, k);
        std::vector<std::vector<uint8_t>> seen(pn);
        std::vector<Sizes> sz(pn);
        for (int j = 0; j < pn; ++j) {
            const FrameArgs& f = D.frames[D.plist[w][j]];
            seen[j].assign((size_t)f.tiles_x * f.tiles_y, 0);
            sz[j] = sizes_of(f);
            CHECK(D.prefix[w][j + 1] - D.prefix[w][j] == (uint32_t)f.tiles_x * f.tiles_y, "frame %d tiles", j);
        }
        uint32_t head[kXcds] = {};
        std::vector<int> qi(wgs, 0), cursor(wgs, 0);
        std::vector<bool> done(wgs, false);
        int active = wgs;
        while (active > 0) {
            for (int g = 0; g < wgs; ++g) {
                if (done[g]) continue;
                const int home = g % kXcds;
                // the next claim of workgroup g: its current run, else the following ones
                for (;;) {
                    if (qi[g] == kXcds) {
                        done[g] = true;
                        --active;
                        break;
                    }
                    const int k = (home + qi[g]) & (kXcds - 1);
                    const uint32_t first = D.split[w][k], count = D.split[w][k + 1] - first;
                    const uint32_t item = head[k]++;
                    if (item >= count) {
                        ++qi[g];
                        continue;
                    }
                    const uint32_t gt = first + item;
                    CHECK(gt < total, "tile %u of %u", gt, total);
                    const int j = batch_frame(D, w, gt, cursor[g]);
                    cursor[g] = j;
                    CHECK(j >= 0 && j < pn && D.prefix[w][j] <= gt && gt < D.prefix[w][j + 1],
                          "cursor: tile %u -> frame %d", gt, j);
                    const FrameArgs& f = D.frames[D.plist[w][j]];
                    int tx, ty;
                    walk(f, gt - D.prefix[w][j], tx, ty);
                    CHECK(tx >= 0 && tx < f.tiles_x && ty >= 0 && ty < f.tiles_y, "batch walk -> (%d, %d)", tx, ty);
                    if (tx >= 0 && tx < f.tiles_x && ty >= 0 && ty < f.tiles_y) {
                        CHECK(seen[j][(size_t)ty * f.tiles_x + tx]++ == 0, "batch tile claimed twice");
                        for (int t = 0; t < 256; ++t) {
                            int x, y, li;
                            tile_pixel(f, tx, ty, t, x, y, li);
                            if (x < f.W && y < f.H) check_pixel(f, sz[j], x, y, li);
                        }
                    }
                    break;  // one claim per turn
                }
            }
        }
        for (int j = 0; j < pn; ++j) {
            long miss = 0;
            for (uint8_t c : seen[j]) miss += c != 1;
            CHECK(miss == 0, "width %d frame %d: %ld tiles not claimed exactly once", w, j, miss);
        }
    }
}


static void emulate_batch(const std::vector<Frame>& frames, LaunchShape shape, int wgs) {
    std::vector<ssvb_frame> F(frames.size());
    std::vector<FrameArgs> A(frames.size());
    for (size_t i = 0; i < frames.size(); ++i) make_frame(frames[i], shape, true, A[i], &F[i]);
    static FrameTables tab;
    tab.forced = true;
    tab.force = shape;
    emulate_batch_frames(F, A, tab, wgs);
}

// ---------------------------------------------------------------------------------------
// fuzz: random frames, cameras, parameters, pitches, formats and launch shapes, each field
// now and then outside what the library accepts.  Every input ssvb_validate accepts is
// run through the index path as above; the rest must be rejected before any kernel.
// ---------------------------------------------------------------------------------------
struct FuzzRng {
    uint64_t s;
    uint64_t next() {  // splitmix64
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int range(int lo, int hi) { return lo + (int)(next() % (uint64_t)(hi - lo + 1)); }  // [lo, hi]
    double uni() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    double logu(double lo, double hi) { return lo * pow(hi / lo, uni()); }
    bool coin(double p) { return uni() < p; }
};

static void fuzz(long n, uint64_t seed, long& accepted, long& rejected, long& emulated, long& batches) {
    FuzzRng R{seed};
    std::vector<ssvb_frame> pending;
    const double bad = 0.02;  // chance of each field being drawn outside the accepted range
    static const int kTilesF[][3] = {{32, 8, 1}, {16, 16, 1}, {64, 4, 1}, {8, 32, 1}, {16, 8, 2}, {8, 16, 2},
                                     {32, 4, 2}, {8, 8, 4},   {16, 4, 4}, {8, 4, 8},  {4, 8, 8},  {7, 9, 3}};
    static FrameTables tab;
    for (long it = 0; it < n; ++it) {
        int W, H;
        switch (R.range(0, 9)) {
            case 0: W = R.range(1, 16384), H = R.range(1, 8); break;  // thin extremes
            case 1: W = R.range(1, 8), H = R.range(1, 16384); break;
            case 2: W = R.range(0, 3), H = R.range(0, 3); break;
            default: W = R.range(1, 420), H = R.range(1, 300); break;
        }
        if (R.coin(bad)) W = R.coin(0.5) ? -R.range(1, 5) : 16385 + R.range(0, 5);
        if (R.coin(bad)) H = R.coin(0.5) ? -R.range(1, 5) : 16385 + R.range(0, 5);
        ssvb_camera cam;
        cam.width = W, cam.height = H;
        cam.fx = (float)R.logu(1e-3, 1e5);
        cam.fy = R.coin(0.5) ? cam.fx : (float)R.logu(1e-3, 1e5);
        cam.cx = (float)((R.uni() * 5.0 - 2.0) * (W > 0 ? W : 1));
        cam.cy = (float)((R.uni() * 5.0 - 2.0) * (H > 0 ? H : 1));
        for (int i = 0; i < 9; ++i) cam.view_to_world[i] = (float)(R.uni() * 2.0 - 1.0);
        if (R.coin(bad)) cam.fx = R.coin(0.5) ? 0.0f : NAN;
        if (R.coin(bad)) cam.cy = INFINITY;
        ssvb_params p;
        ssvb_default_params(&p);
        p.slices = R.coin(0.8) ? R.range(1, 8) : R.range(1, 64);
        p.steps = R.coin(0.7) ? R.range(1, 32) : R.range(1, 1024);
        p.sectors = R.coin(0.5) ? 32 : 128;
        {
            static const int na[] = {1, 2, 4, 8, 16, 32};
            p.ambient_samples = na[R.range(0, 5)];
        }
        p.radius = (float)R.logu(1e-4, 1e9);
        p.thickness = R.coin(0.2) ? INFINITY : (float)(R.uni() * 2.0);
        p.thickness_slope = R.coin(0.5) ? 0.0f : (float)(R.uni() * 0.2);
        p.max_radius_px = R.coin(0.5) ? 0.0f : (float)R.logu(0.01, 40000.0);
        p.min_step_q4 = R.range(1, 16);
        p.step_distribution = R.range(0, 1);
        p.resolution = R.range(1, 2);
        p.hit_criterion = R.range(0, 1);
        p.noise = R.range(0, 2);
        p.seed = (uint32_t)R.next();
        if (R.coin(bad)) p.slices = R.coin(0.5) ? 0 : 65;
        if (R.coin(bad)) p.steps = R.coin(0.5) ? 0 : 1025;
        if (R.coin(bad)) p.sectors = R.coin(0.5) ? 64 : 0;
        if (R.coin(bad)) p.ambient_samples = R.coin(0.5) ? 3 : 64;
        if (R.coin(bad)) p.radius = R.coin(0.5) ? -1.0f : NAN;
        if (R.coin(bad)) p.max_radius_px = -1.0f;
        if (R.coin(bad)) p.min_step_q4 = R.coin(0.5) ? 0 : 17;
        if (R.coin(bad)) p.resolution = 3;
        // inputs: formats, channels and pitches (padded rows, some spanning close to 4 GiB)
        auto image = [&](uintptr_t base, bool depth) {
            ssvb_image im;
            const bool f16 = !depth && R.coin(0.5);
            im.dtype = f16 ? SSVB_F16 : SSVB_F32;
            im.channels = depth ? 1 : (R.coin(0.5) ? 3 : 4);
            const int64_t es = f16 ? 2 : 4;
            const int64_t row = (int64_t)(W > 0 ? W : 0) * im.channels * es;
            im.ptr = (const void*)base;
            switch (R.range(0, 3)) {
                case 0: im.pitch_bytes = 0; break;
                case 1: im.pitch_bytes = row + es * R.range(0, 64); break;
                case 2: {  // as wide as the 4 GiB span allows
                    const int64_t hmax = H > 1 ? H - 1 : 1;
                    const int64_t room = ((int64_t)1 << 32) - row;
                    int64_t pitch = room / hmax;
                    pitch -= pitch % es;
                    im.pitch_bytes = pitch >= row ? pitch - es * R.range(0, 3) : 0;
                    if (im.pitch_bytes < row) im.pitch_bytes = 0;
                    break;
                }
                default: im.pitch_bytes = row + es * R.range(0, 4096); break;
            }
            if (R.coin(bad)) im.pitch_bytes = row > es ? row - es : row + 1;
            if (R.coin(bad)) im.ptr = (const void*)(base + 1);
            if (R.coin(bad)) im.channels = depth ? 3 : 5;
            if (R.coin(bad)) im.dtype = depth ? SSVB_F16 : (ssvb_dtype)7;
            return im;
        };
        const ssvb_image depth = image(0x10000000ull, true);
        const ssvb_image normal = image(0x1000000000ull, false);
        const ssvb_image radiance = image(0x2000000000ull, false);
        const bool masks = R.coin(0.4) && (p.resolution == 1 || R.coin(bad));  // no masks at half resolution
        auto opitch = [&](int64_t row) -> int64_t {
            if (R.coin(bad)) return row + 2;
            return R.coin(0.5) ? 0 : row + 4 * R.range(0, 256);
        };
        const int64_t Wc = W > 0 ? W : 0;
        ssvb_outputs o{(float*)0x3000000000ull, (float*)0x4000000000ull, (float*)0x5000000000ull,
                       masks ? (uint32_t*)0x6000000000ull : nullptr, opitch(Wc * 4), opitch(Wc * 12), opitch(Wc * 12),
                       masks ? opitch(Wc * (p.slices > 0 ? p.slices : 1) * (p.sectors > 0 ? p.sectors / 32 : 1) * 4)
                             : 0};
        const int ti = R.range(0, 11);
        tab.forced = R.coin(0.7);
        tab.force = LaunchShape{kTilesF[ti][0], kTilesF[ti][1], R.range(0, 9), kTilesF[ti][2]};
        if (ssvb_validate(&depth, &normal, &radiance, &cam, &p, &o) != SSVB_OK) {
            ++rejected;
            continue;
        }
        ++accepted;
        if ((int64_t)W * H == 0) continue;
        FrameArgs A;
        fill_frame(A, &tab, &depth, &normal, &radiance, &cam, &p, &o);
        CHECK(A.tile_w * A.tile_h * A.lp == 256 && A.strip >= 1 && A.strip <= (A.tiles_x > 0 ? A.tiles_x : 1),
              "launch shape %dx%d lp %d strip %d", A.tile_w, A.tile_h, A.lp, A.strip);
        check_lattice(A);
        if ((int64_t)W * H <= 300000) {
            emulate_frame(A);
            ++emulated;
            emulate_slices(A, (p.seed & 7) == 7 ? 65536u : 1u + (p.seed >> 8) % 300u);
        }
        {
            const Sizes S = sizes_of(A);
            const int64_t cap = 16 << 20;  // real buffers only for spans of at most 16 MB
            if ((int64_t)W * H <= 20000 && S.depth <= cap && S.normal <= cap && S.ao <= cap && S.gi <= cap &&
                S.amb <= cap) {
                if (A.sub == 2) g_upsampled += check_upsample(A);
                g_denoised += check_denoise(A);
            }
        }
        // small frames also go into batches of up to kMaxBatch, as ssvb_compute_batch packs
        // them (frames of at most kPackTiles tiles), under one context launch shape
        if ((uint32_t)A.tiles_x * (uint32_t)A.tiles_y <= kPackTiles && (int64_t)W * H <= 60000) {
            pending.push_back(ssvb_frame{depth, normal, radiance, cam, p, o});
            if ((int)pending.size() == R.range(1, kMaxBatch) || (int)pending.size() == kMaxBatch) {
                static FrameTables btab;
                const int bi = R.range(0, 11);
                btab.forced = R.coin(0.7);
                btab.force = LaunchShape{kTilesF[bi][0], kTilesF[bi][1], R.range(0, 9), kTilesF[bi][2]};
                std::vector<FrameArgs> BA(pending.size());
                for (size_t i = 0; i < pending.size(); ++i) {
                    const ssvb_frame& f = pending[i];
                    fill_frame(BA[i], &btab, &f.depth, &f.normal, &f.radiance, &f.camera, &f.params, &f.out);
                }
                // the packed list holds only frames small enough under this shape
                std::vector<ssvb_frame> keep;
                std::vector<FrameArgs> keepA;
                for (size_t i = 0; i < pending.size(); ++i)
                    if ((uint32_t)BA[i].tiles_x * (uint32_t)BA[i].tiles_y <= kPackTiles) {
                        keep.push_back(pending[i]);
                        keepA.push_back(BA[i]);
                    }
                static const int kWgs[] = {1, 7, 1024};
                emulate_batch_frames(keep, keepA, btab, kWgs[R.range(0, 2)]);
                ++batches;
                pending.clear();
            }
        }
    }
}

int main(int argc, char** argv) {
    bool quick = false;
    int part_k = 0, part_n = 1;  // --part k/n: every n-th frame shape from the k-th (batches in the last)
    long fuzz_n = 0;
    uint64_t fuzz_seed = 1;
    for (int i = 1; i < argc; ++i) {
        if (!strcmp(argv[i], "--interleaved")) g_interleaved = true;
        if (!strcmp(argv[i], "--quick")) quick = true;
        if (!strcmp(argv[i], "--part") && i + 1 < argc) sscanf(argv[i + 1], "%d/%d", &part_k, &part_n);
        if (!strcmp(argv[i], "--fuzz") && i + 2 < argc) {
            fuzz_n = atol(argv[i + 1]);
            fuzz_seed = strtoull(argv[i + 2], nullptr, 10);
        }
    }
    if (fuzz_n > 0) {
        long acc = 0, rej = 0, emu = 0, bat = 0;
        fuzz(fuzz_n, fuzz_seed, acc, rej, emu, bat);
        printf("fuzz: %ld inputs, %ld accepted (%ld emulated), %ld rejected, %ld batches, %ld slice-major items, "
               "%ld upsampled and %ld denoised cells on real buffers, %ld checks, %ld failed\n",
               fuzz_n, acc, emu, rej, bat, g_slice_items, g_upsampled, g_denoised, g_checks, g_fail);
        return g_fail != 0;
    }
    // the launch shapes of the autotuner (tile w, h, lanes) x strips, and the default
    static const int kTiles[][3] = {{32, 8, 1}, {16, 16, 1}, {64, 4, 1}, {8, 32, 1}, {16, 8, 2}, {8, 16, 2},
                                    {32, 4, 2}, {8, 8, 4},   {16, 4, 4}, {8, 4, 8},  {4, 8, 8}};
    static const int kStrips[] = {1, 2, 3, 4, 8};
    // frames of the GPU suite: workloads, tests, batch and serving mixes, ragged and extreme
    // sizes (W, H, slices, steps, sectors, resolution, distribution, fp16, channels, pad, masks)
    struct Spec {
        int W, H, nd, ns, nb, sub, dist, f16, ch, pad, masks;
    };
    std::vector<Spec> specs = {
        {128, 128, 2, 8, 32, 1, 0, 0, 3, 0, 1},   {64, 48, 4, 8, 32, 1, 0, 0, 3, 0, 1},
        {67, 45, 3, 5, 32, 1, 0, 0, 3, 0, 1},     {1, 1, 3, 5, 32, 1, 0, 0, 3, 0, 1},
        {1, 37, 3, 5, 32, 1, 0, 1, 4, 0, 1},      {37, 1, 3, 5, 32, 1, 0, 0, 4, 0, 1},
        {129, 3, 3, 5, 128, 1, 0, 0, 3, 0, 1},    {200, 113, 4, 16, 32, 1, 0, 1, 3, 3, 0},
        {33, 91, 8, 3, 32, 1, 0, 0, 4, 0, 1},     {96, 64, 5, 7, 32, 1, 0, 0, 3, 5, 1},
        {160, 90, 7, 9, 32, 1, 1, 1, 3, 0, 0},    {39, 23, 64, 2, 128, 1, 0, 0, 3, 0, 1},
        {41, 31, 3, 1024, 32, 1, 1, 0, 3, 0, 1},  {65, 33, 4, 16, 32, 2, 0, 0, 3, 0, 0},
        {255, 143, 4, 16, 128, 2, 1, 1, 4, 7, 0}, {256, 144, 2, 8, 32, 1, 0, 0, 3, 0, 0},
        {320, 180, 4, 16, 32, 1, 0, 0, 3, 0, 0},  {480, 270, 2, 16, 32, 1, 0, 0, 3, 0, 0},
        {640, 360, 4, 8, 32, 1, 0, 0, 3, 0, 0},   {960, 540, 8, 32, 32, 1, 0, 1, 3, 0, 0},
        {1280, 720, 2, 8, 32, 1, 0, 0, 3, 0, 0},  {1920, 1080, 4, 16, 32, 1, 0, 0, 3, 0, 1},
        {1920, 1080, 4, 16, 128, 2, 1, 0, 3, 0, 0}, {2560, 1440, 8, 32, 32, 1, 0, 0, 3, 0, 0},
        {3840, 2160, 8, 32, 32, 1, 0, 1, 3, 0, 1}, {16384, 1, 3, 2, 32, 1, 0, 0, 3, 0, 1},
        {1, 16384, 3, 2, 32, 1, 0, 0, 3, 0, 1},   {3, 4099, 3, 2, 32, 1, 0, 0, 3, 0, 1},
    };
    auto frame_of = [](const Spec& s, bool masks) {
        Frame f;
        f.W = s.W, f.H = s.H, f.nd = s.nd, f.ns = s.ns, f.nb = s.nb, f.sub = s.sub, f.dist = s.dist;
        f.min_q4 = s.ns >= 1024 ? 1 : 16;
        f.n16 = f.r16 = s.f16 != 0;
        f.nch = f.rch = s.ch;
        f.pad = s.pad;
        f.masks = masks && s.sub == 1;
        f.radius = (s.W == 1 || s.H == 1 || s.W == 3) ? 1e9f : 3.0f;  // the extreme-size tests' reach
        return f;
    };
    long frames_done = 0;
    for (size_t si = 0; si < specs.size(); ++si) {
        if ((int)(si % (size_t)part_n) != part_k) continue;
        const Spec& s = specs[si];
        const Frame f = frame_of(s, s.masks != 0);
        const bool big = (int64_t)s.W * s.H > 2000000;
        for (const auto& tl : kTiles) {
            for (int st : kStrips) {
                if ((big || quick) && !(st == 1 || st == 2 || st == 4)) continue;
                if ((big || quick) && !(tl[2] == 1 || (tl[0] == 16 && tl[1] == 8))) continue;
                FrameArgs A;
                make_frame(f, LaunchShape{tl[0], tl[1], st, tl[2]}, true, A);
                emulate_frame(A);
                ++frames_done;
            }
        }
        // the library's default shape (no forced shape)
        FrameArgs A;
        make_frame(f, LaunchShape{32, 8, 4, 1}, false, A);
        emulate_frame(A);
        check_lattice(A);
        ++frames_done;
        // the slice-major order over chunks of 1, 7 and 64 tiles and one chunk of everything
        if (!g_interleaved) {
            for (uint32_t c : {1u, 7u, 64u, 65536u}) {
                if (big && c != 64u) continue;
                emulate_slices(A, c);
            }
            FrameArgs A2;  // and from a launch shape with lanes per pixel
            make_frame(f, LaunchShape{8, 8, 3, 4}, true, A2);
            emulate_slices(A2, 5u);
        }
        // the half-resolution fill and the denoiser on real buffers of the frame's spans
        if ((int64_t)s.W * s.H <= 400000 && !g_interleaved) {  // independent of the walk
            if (A.sub == 2) g_upsampled += check_upsample(A);
            g_denoised += check_denoise(A);
        }
    }
    // batches: the mixed small frames of the GPU batch tests, with every launch shape
    std::vector<Frame> batch;
    for (const Spec& s : specs) {
        if ((int64_t)s.W * s.H > 400000) continue;
        batch.push_back(frame_of(s, false));
    }
    for (int i = 0; i < 40; ++i) {  // one-tile frames up to a few tiles, as the packed-batch tests draw
        const Spec s{1 + (i * 7) % 39, 1 + (i * 5) % 23, 2 + i % 3, 8, (i % 4 == 3) ? 128 : 32, 1 + (i % 5 == 4), 0,
                     i % 2, 3, 0, 0};
        batch.push_back(frame_of(s, false));
    }
    if (batch.size() > (size_t)kMaxBatch) batch.resize(kMaxBatch);
    long batches = 0;
    for (const auto& tl : kTiles) {
        for (int st : kStrips) {
            if ((quick && st != 4) || part_k != part_n - 1) continue;
            for (int wgs : {1, 7, 1024}) {
                emulate_batch(batch, LaunchShape{tl[0], tl[1], st, tl[2]}, wgs);
                ++batches;
            }
        }
    }
    printf("%s walk: %ld frame launches, %ld batches, %ld slice-major items, %ld upsampled and %ld denoised cells "
           "on real buffers, %ld checks, %ld failed\n",
           g_interleaved ? "interleaved" : "strip", frames_done, batches, g_slice_items, g_upsampled, g_denoised,
           g_checks, g_fail);
    return g_fail != 0;
}
