// Edge-aware a-trous denoising of the gather's outputs: kernel arguments and launcher.
#ifndef SSVB_DENOISE_H
#define SSVB_DENOISE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssvb {

// One pass: reads the AO / GI / ambient images `in_*`, writes `out_*` (never the same
// memory).  The pass runs on a grid of cells: every pixel (g = 1) or the pixels with both
// coordinates even (g = 2); cell (u, v) is pixel (g u, g v).
struct DenoiseArgs {
    const float* depth;
    const char* normal;
    int64_t depth_pitch, normal_pitch;   // bytes
    int32_t normal_ch, normal_f16;
    const float* in_ao;
    const float* in_gi;
    const float* in_amb;
    int64_t in_ao_pitch, in_gi_pitch, in_amb_pitch;
    float* out_ao;
    float* out_gi;
    float* out_amb;
    int64_t out_ao_pitch, out_gi_pitch, out_amb_pitch;
    int32_t W, H;          // image
    int32_t g;             // cell stride in pixels, 1 or 2
    int32_t gw, gh;        // cells per row and column
    int32_t tiles_x;       // 16 x 16-cell output tiles per row
    int32_t tiles;         // tiles in all
    float cx, cy, inv_fx, inv_fy;
    float inv_sigma;       // 1 / plane_sigma (0: no plane term)
    int32_t normal_power;  // k of max(0, n_p . n_q)^k
};

constexpr int kDenoiseTile = 16;

// Pass `pass` (taps 2^pass cells apart; pass < 3) on `stream`.
hipError_t launch_denoise(const DenoiseArgs& D, int pass, hipStream_t stream);

}  // namespace ssvb

#endif
