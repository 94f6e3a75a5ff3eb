// Host build of the gather's per-pixel code (csrc/ssvb_pixel.h), for the CPU test suite.
//
// host_gather() runs, on the CPU, the same per-pixel functions the gfx950 kernels run
// (gather_pixel, and upsample_pixel at half resolution) on every computed pixel of a frame
// in host memory, one lane per pixel, with the frame constants and tables the library
// itself derives (fill_frame, fill_tables from libssvb.so).  The template instance is the
// one the library's single-frame launcher picks for the frame's mode, or with `generic`
// the run-time-dispatch instance the batch kernel uses.  Only the device primitives differ
// from the GPU: the hardware reciprocal (about 1 ulp) is an exact division here, and the
// compiler may contract differently, so results match the GPU to FP32 rounding, not bit
// for bit.
#include <math.h>
#include <string.h>

#include <vector>

#include "ssvb_host.h"
#include "ssvb_pixel.h"

using namespace ssvb;

namespace {

ExactLds g_lds;  // slot 0 is the one lane's

template <int CRIT, bool TINF, int FMT, int NB>
void run_pixels(const FrameArgs& A) {
    for (int y = 0; y < A.H; y += A.sub)
        for (int x = 0; x < A.W; x += A.sub)
            gather_pixel<CRIT, MODE_COMPUTE, TINF, FMT, NB>(A, g_lds, x, y, 0, 1, nullptr, nullptr);
}

template <int CRIT, bool TINF>
void run_fmt(const FrameArgs& A) {
    switch (A.normal_f16 | (A.radiance_f16 << 1)) {
        case 0: run_pixels<CRIT, TINF, 0, 32>(A); break;
        case 1: run_pixels<CRIT, TINF, 1, 32>(A); break;
        case 2: run_pixels<CRIT, TINF, 2, 32>(A); break;
        default: run_pixels<CRIT, TINF, 3, 32>(A); break;
    }
}

}  // namespace

extern "C" int host_gather(const ssvb_image* depth, const ssvb_image* normal, const ssvb_image* radiance,
                           const ssvb_camera* camera, const ssvb_params* params, const ssvb_outputs* out,
                           int generic) {
    const ssvb_status s = ssvb_validate(depth, normal, radiance, camera, params, out);
    if (s != SSVB_OK) return (int)s;
    if ((int64_t)camera->width * camera->height == 0) return 0;
    static int2 lut[kLutSize];
    static double2 half[129], half128[513];
    fill_tables(lut, half, half128);
    FrameTables tab;
    tab.d_lut = lut;
    tab.d_half = half;
    tab.d_half128 = half128;
    FrameArgs A;
    fill_frame(A, &tab, depth, normal, radiance, camera, params, out);
    const bool tinf = isinf(A.t0);
    // the instance the library launches for this frame (launch_plain), or the batch kernel's
    if (A.nb == 128) {
        if (!generic && A.criterion == SSVB_HIT_ROUND && !tinf && !A.normal_f16 && !A.radiance_f16)
            run_pixels<SSVB_HIT_ROUND, false, 0, 128>(A);
        else
            run_pixels<-1, false, -1, 128>(A);
    } else if (generic) {
        run_pixels<-1, false, -1, 32>(A);
    } else if (A.criterion == SSVB_HIT_ROUND) {
        if (tinf) run_fmt<SSVB_HIT_ROUND, true>(A);
        else run_fmt<SSVB_HIT_ROUND, false>(A);
    } else {
        if (tinf) run_fmt<SSVB_HIT_PSEUDOCODE, true>(A);
        else run_fmt<SSVB_HIT_PSEUDOCODE, false>(A);
    }
    if (A.sub == 2)
        for (int y = 0; y < A.H; ++y)
            for (int x = 0; x < A.W; ++x) upsample_pixel(A, x, y);
    return 0;
}

// The slice-major order of a frame on host buffers, as gather_slices and reduce_slices run
// it: the items of each XCD's run in the kernel's order (slice_item over chunks of `chunk`
// tiles, the strip walk, one lane per pixel), each running one slice of its tile's pixels
// into a partial buffer, then the reduction of every computed pixel and, at half
// resolution, the fill.  Returns 0, or the validation status.
template <int NB>
static void run_slices(const FrameArgs& A, float* partial, uint32_t chunk) {
    const uint32_t nt = (uint32_t)A.tiles_x * (uint32_t)A.tiles_y;
    for (int k = 0; k < kXcds; ++k) {
        uint32_t first, count;
        xcd_run(nt, k, first, count);
        for (uint32_t j = 0; j < count * (uint32_t)A.nd; ++j) {
            uint32_t tile;
            int slice, tx, ty;
            slice_item(chunk, A.nd, count, j, tile, slice);
            walk_tile(A, first + tile, tx, ty);
            for (int t = 0; t < 256; ++t) {
                int x, y, li;
                tile_pixel(A, tx, ty, t, x, y, li);
                if ((unsigned)x < (unsigned)A.W && (unsigned)y < (unsigned)A.H)
                    gather_pixel<-1, MODE_PARTIAL, false, -1, NB>(A, g_lds, x, y, slice, A.nd, nullptr, partial);
            }
        }
    }
}

extern "C" int host_gather_slices(const ssvb_image* depth, const ssvb_image* normal, const ssvb_image* radiance,
                                  const ssvb_camera* camera, const ssvb_params* params, const ssvb_outputs* out,
                                  int chunk) {
    const ssvb_status s = ssvb_validate(depth, normal, radiance, camera, params, out);
    if (s != SSVB_OK) return (int)s;
    if ((int64_t)camera->width * camera->height == 0) return 0;
    static int2 lut[kLutSize];
    static double2 half[129], half128[513];
    fill_tables(lut, half, half128);
    FrameTables tab;
    tab.d_lut = lut;
    tab.d_half = half;
    tab.d_half128 = half128;
    FrameArgs A;
    fill_frame(A, &tab, depth, normal, radiance, camera, params, out);
    if (A.lp > 1) set_launch(A, LaunchShape{A.tile_w * A.lp, A.tile_h, A.strip, 1});
    const size_t gw = (size_t)(A.W + A.sub - 1) / A.sub, gh = (size_t)(A.H + A.sub - 1) / A.sub;
    std::vector<float> partial(gw * gh * (size_t)A.nd * kPartialFloats, NAN);
    if (A.nb == 128) run_slices<128>(A, partial.data(), (uint32_t)chunk);
    else run_slices<32>(A, partial.data(), (uint32_t)chunk);
    for (size_t v = 0; v < gh; ++v)
        for (size_t u = 0; u < gw; ++u) reduce_pixel(A, partial.data(), (int)u * A.sub, (int)v * A.sub);
    if (A.sub == 2)
        for (int y = 0; y < A.H; ++y)
            for (int x = 0; x < A.W; ++x) upsample_pixel(A, x, y);
    return 0;
}

// The FP32 sector arguments of every sample of a frame (the endpoint hook's instances, at
// 32 or 128 sectors), for the error bound behind the exact decision's guard band: ep holds
// W * H * N_d * 2 * N_s * 2 floats per pixel, slice, side (+ then -), step and argument,
// left as the caller filled them for skipped samples.  Returns 0, or the validation status.
template <int CRIT, int NB>
static void run_endpoints(const FrameArgs& A, float* ep) {
    const int64_t per = (int64_t)A.nd * 2 * A.ns * 2;
    for (int y = 0; y < A.H; ++y)
        for (int x = 0; x < A.W; ++x) {
            float* d = ep + ((int64_t)y * A.W + x) * per;
            if (A.normal_f16) gather_pixel<CRIT, MODE_ENDPOINTS, false, 1, NB>(A, g_lds, x, y, 0, 1, nullptr, d);
            else gather_pixel<CRIT, MODE_ENDPOINTS, false, 0, NB>(A, g_lds, x, y, 0, 1, nullptr, d);
        }
}

extern "C" int host_endpoints(const ssvb_image* depth, const ssvb_image* normal, const ssvb_image* radiance,
                              const ssvb_camera* camera, const ssvb_params* params, const ssvb_outputs* out,
                              float* ep) {
    const ssvb_status s = ssvb_validate(depth, normal, radiance, camera, params, out);
    if (s != SSVB_OK) return (int)s;
    if ((int64_t)camera->width * camera->height == 0) return 0;
    static int2 lut[kLutSize];
    static double2 half[129], half128[513];
    fill_tables(lut, half, half128);
    FrameTables tab;
    tab.d_lut = lut;
    tab.d_half = half;
    tab.d_half128 = half128;
    FrameArgs A;
    fill_frame(A, &tab, depth, normal, radiance, camera, params, out);
    const bool round = A.criterion == SSVB_HIT_ROUND;
    if (A.nb == 128) {
        if (round) run_endpoints<SSVB_HIT_ROUND, 128>(A, ep);
        else run_endpoints<SSVB_HIT_PSEUDOCODE, 128>(A, ep);
    } else {
        if (round) run_endpoints<SSVB_HIT_ROUND, 32>(A, ep);
        else run_endpoints<SSVB_HIT_PSEUDOCODE, 32>(A, ep);
    }
    return 0;
}

// atan2_pos, the kernels' FP32 arc tangent for y >= 0, on n argument pairs.
extern "C" void host_atan2(const float* y, const float* x, float* out, int64_t n) {
    for (int64_t i = 0; i < n; ++i) out[i] = atan2_pos(y[i], x[i]);
}

// The visibility-mask primitives at N_b = 32, 64 or 128 sectors, for exhaustive checks:
// host_mask_range writes mask_range(a, b)'s N_b / 32 words; host_mask_cover ORs the ranges
// [a[j], b[j]) into an empty mask in order with cover(), writing each step's newly covered
// count and the final words and count.  Return 0, or -1 for another N_b.
template <int NB>
static void mask_range_words(int a, int b, uint32_t* out) {
    const SMask<NB> m = mask_range<NB>(a, b);
    for (int i = 0; i < SMask<NB>::W; ++i) out[i] = m.w[i];
}

template <int NB>
static void mask_cover_run(const int* a, const int* b, int n, int* fresh, uint32_t* words, int* count) {
    SMask<NB> B = mask_none<NB>();
    for (int j = 0; j < n; ++j) fresh[j] = cover<NB>(B, mask_range<NB>(a[j], b[j]));
    for (int i = 0; i < SMask<NB>::W; ++i) words[i] = B.w[i];
    *count = NB == 32 ? popc32(B.w[0]) : B.n;
}

extern "C" int host_mask_range(int nb, int a, int b, uint32_t* out) {
    switch (nb) {
        case 32: mask_range_words<32>(a, b, out); return 0;
        case 64: mask_range_words<64>(a, b, out); return 0;
        case 128: mask_range_words<128>(a, b, out); return 0;
        default: return -1;
    }
}

extern "C" int host_mask_cover(int nb, const int* a, const int* b, int n, int* fresh, uint32_t* words,
                               int* count) {
    switch (nb) {
        case 32: mask_cover_run<32>(a, b, n, fresh, words, count); return 0;
        case 64: mask_cover_run<64>(a, b, n, fresh, words, count); return 0;
        case 128: mask_cover_run<128>(a, b, n, fresh, words, count); return 0;
        default: return -1;
    }
}
