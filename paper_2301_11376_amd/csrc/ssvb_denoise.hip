// Edge-aware a-trous denoising of AO, GI and ambient (the denoising pass that Section 4.1
// and Table 2 time after the gather; the paper does not describe it, so this filter is
// this library's own).
//
// Pass i averages each foreground cell over the 5 x 5 taps 2^i cells apart with weights
// h_a h_b exp(-(n_p . (P_q - P_p) / (sigma z_p))^2) max(0, n_p . n_q)^k, h = (1, 4, 6, 4,
// 1) / 16; the centre weighs h_0^2; taps off the image or on background are left out and
// the weights renormalised; a background cell keeps its input.
//
// One workgroup per 16 x 16-cell output tile.  The tile and its apron of 2 * 2^i cells
// are staged once in LDS (view-space position, unit normal, the seven signal channels),
// so every tap is an LDS read (48 bytes); the pass is bound by VALU issue and LDS reads.
#include <hip/hip_runtime.h>

#include "ssvb_denoise.h"
#include "ssvb_denoise_cell.h"

namespace ssvb {
namespace {

constexpr int kThreads = kDenoiseTile * kDenoiseTile;

template <int S, int K2>
__global__ __launch_bounds__(kThreads) void denoise_pass(DenoiseArgs D) {
    constexpr int E = kDenoiseTile + 4 * S;  // staged tile edge, cells
    constexpr int N = E * E;
    __shared__ float4 sA[N];  // depth (0 off the image or on background), unit normal xyz
    __shared__ float4 sB[N];  // AO, GI rgb
    __shared__ float4 sC[N];  // ambient rgb, unused
    // workgroup b runs on XCD b mod 8: give each XCD one contiguous run of tiles (rows of
    // tiles, so that the aprons it stages overlap in its own L2)
    const int run = (D.tiles + 7) / 8;
    const int tile = ((int)blockIdx.x % 8) * run + (int)blockIdx.x / 8;
    if (tile >= D.tiles) return;
    const int u0 = (tile % D.tiles_x) * kDenoiseTile - 2 * S;
    const int v0 = (tile / D.tiles_x) * kDenoiseTile - 2 * S;

    for (int i = (int)threadIdx.x; i < N; i += kThreads) {
        const int u = u0 + i % E, v = v0 + i / E;
        float4 A = make_float4(0.0f, 0.0f, 0.0f, 0.0f), B = A, C = A;
        if (u >= 0 && v >= 0 && u < D.gw && v < D.gh) dn::stage_cell(D, u, v, A, B, C);
        sA[i] = A;
        sB[i] = B;
        sC[i] = C;
    }
    __syncthreads();

    dn::filter_cell<S, K2>(D, sA, sB, sC, u0, v0, (int)threadIdx.x % kDenoiseTile, (int)threadIdx.x / kDenoiseTile);
}

template <int S>
void launch_pass(const DenoiseArgs& D, hipStream_t stream) {
    const int grid = 8 * ((D.tiles + 7) / 8);  // whole runs, one per XCD
    if (D.normal_power == 16)
        hipLaunchKernelGGL((denoise_pass<S, 4>), dim3(grid), dim3(kThreads), 0, stream, D);
    else
        hipLaunchKernelGGL((denoise_pass<S, -1>), dim3(grid), dim3(kThreads), 0, stream, D);
}

}  // namespace

hipError_t launch_denoise(const DenoiseArgs& D, int pass, hipStream_t stream) {
    if (D.tiles <= 0) return hipSuccess;
    switch (pass) {
        case 0: launch_pass<1>(D, stream); break;
        case 1: launch_pass<2>(D, stream); break;
        case 2: launch_pass<4>(D, stream); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ssvb
