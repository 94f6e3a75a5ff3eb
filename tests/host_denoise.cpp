// Host build of the denoiser's per-cell code (csrc/ssvb_denoise_cell.h), for the CPU test
// suite.
//
// host_denoise() runs, on the CPU, what ssvb_denoise runs on the device: for each pass the
// library's own pass arguments (fill_denoise), every 16 x 16-cell tile staged with
// stage_cell and every output cell filtered with filter_cell (the kernel's template
// instance: taps 2^pass cells apart, normal power 16 by squarings or any power by
// square-and-multiply); at half resolution the upsampler of the gather (upsample_pixel)
// afterwards.  Only the device primitives differ from the GPU: the hardware reciprocal
// square root, exp2 and reciprocal are exact functions here.
#include <math.h>
#include <string.h>

#include <vector>

#include "ssvb_denoise_cell.h"
#include "ssvb_host.h"
#include "ssvb_pixel.h"

using namespace ssvb;

namespace {

template <int S, int K2>
void run_pass(const DenoiseArgs& D) {
    constexpr int E = kDenoiseTile + 4 * S, N = E * E;
    std::vector<float4> sA(N), sB(N), sC(N);
    for (int tile = 0; tile < D.tiles; ++tile) {
        const int u0 = (tile % D.tiles_x) * kDenoiseTile - 2 * S;
        const int v0 = (tile / D.tiles_x) * kDenoiseTile - 2 * S;
        for (int i = 0; i < N; ++i) {
            const int u = u0 + i % E, v = v0 + i / E;
            float4 A = make_float4(0.0f, 0.0f, 0.0f, 0.0f), B = A, C = A;
            if (u >= 0 && v >= 0 && u < D.gw && v < D.gh) dn::stage_cell(D, u, v, A, B, C);
            sA[i] = A;
            sB[i] = B;
            sC[i] = C;
        }
        for (int t = 0; t < kDenoiseTile * kDenoiseTile; ++t)
            dn::filter_cell<S, K2>(D, sA.data(), sB.data(), sC.data(), u0, v0, t % kDenoiseTile, t / kDenoiseTile);
    }
}

template <int S>
void run_pass_k(const DenoiseArgs& D) {
    if (D.normal_power == 16) run_pass<S, 4>(D);
    else run_pass<S, -1>(D);
}

}  // namespace

// The denoiser on host buffers, as ssvb_denoise runs it (the caller passes valid inputs;
// `tmp` may be NULL for one pass).  Returns 0.
extern "C" int host_denoise(const ssvb_image* depth, const ssvb_image* normal, const ssvb_camera* camera,
                            const ssvb_outputs* in, const ssvb_outputs* tmp, const ssvb_outputs* out,
                            const ssvb_denoise_params* dp) {
    const ssvb_outputs* src = in;
    DenoiseArgs D;
    for (int i = 0; i < dp->passes; ++i) {
        const ssvb_outputs* dst = ((dp->passes - 1 - i) % 2 == 0) ? out : tmp;
        fill_denoise(D, depth, normal, camera, dp, src, dst);
        if (i == 0) run_pass_k<1>(D);
        else if (i == 1) run_pass_k<2>(D);
        else run_pass_k<4>(D);
        src = dst;
    }
    if (dp->resolution == 2) {
        FrameArgs A;
        fill_upsample(A, depth, camera, out);
        for (int y = 0; y < A.H; ++y)
            for (int x = 0; x < A.W; ++x) upsample_pixel(A, x, y);
    }
    return 0;
}
