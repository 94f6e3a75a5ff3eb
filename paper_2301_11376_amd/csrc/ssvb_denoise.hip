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
#include <math.h>

#include "ssvb_denoise.h"

#define GMEM __attribute__((address_space(1)))

namespace ssvb {
namespace {

constexpr int kThreads = kDenoiseTile * kDenoiseTile;

__device__ __forceinline__ bool foreground(float z) { return z > 0.0f && z < INFINITY; }

__device__ __forceinline__ float ipow(float c, int k) {
    float r = 1.0f;
    for (int e = k; e != 0; e >>= 1) {
        if (e & 1) r *= c;
        c *= c;
    }
    return r;
}

// c^k: K2 >= 0 means k = 2^K2 (K2 squarings), else the general square-and-multiply
template <int K2>
__device__ __forceinline__ float normal_weight(float c, int k) {
    if (K2 < 0) return ipow(c, k);
#pragma unroll
    for (int i = 0; i < (K2 < 0 ? 0 : K2); ++i) c *= c;
    return c;
}

constexpr float kSqrtLog2e = 1.20112240878644980f;  // sqrt(log2(e)): exp(-d^2) = 2^-(d sqrt(log2 e))^2

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
        if (u >= 0 && v >= 0 && u < D.gw && v < D.gh) {
            const int x = u * D.g, y = v * D.g;
            const float z = *(const GMEM float*)((const GMEM char*)D.depth + (int64_t)y * D.depth_pitch + 4 * (int64_t)x);
            if (foreground(z)) {
                const GMEM char* nb = (const GMEM char*)D.normal + (int64_t)y * D.normal_pitch;
                float nx, ny, nz;
                if (D.normal_f16) {
                    const GMEM _Float16* p = (const GMEM _Float16*)nb + (int64_t)x * D.normal_ch;
                    nx = (float)p[0], ny = (float)p[1], nz = (float)p[2];
                } else {
                    const GMEM float* p = (const GMEM float*)nb + (int64_t)x * D.normal_ch;
                    nx = p[0], ny = p[1], nz = p[2];
                }
                const float l2 = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
                const float il = l2 > 0.0f ? __builtin_amdgcn_rsqf(l2) : 0.0f;
                A = make_float4(z, nx * il, ny * il, nz * il);
                const GMEM float* gi = (const GMEM float*)((const GMEM char*)D.in_gi + (int64_t)y * D.in_gi_pitch) + 3 * (int64_t)x;
                const GMEM float* am = (const GMEM float*)((const GMEM char*)D.in_amb + (int64_t)y * D.in_amb_pitch) + 3 * (int64_t)x;
                B = make_float4(*(const GMEM float*)((const GMEM char*)D.in_ao + (int64_t)y * D.in_ao_pitch + 4 * (int64_t)x),
                                gi[0], gi[1], gi[2]);
                C = make_float4(am[0], am[1], am[2], 0.0f);
            }
        }
        sA[i] = A;
        sB[i] = B;
        sC[i] = C;
    }
    __syncthreads();

    const int lx = (int)threadIdx.x % kDenoiseTile, ly = (int)threadIdx.x / kDenoiseTile;
    const int u = u0 + 2 * S + lx, v = v0 + 2 * S + ly;
    if (u >= D.gw || v >= D.gh) return;
    const int x = u * D.g, y = v * D.g;
    const int c = (ly + 2 * S) * E + lx + 2 * S;
    const float4 Ap = sA[c];
    float r[7];
    if (Ap.x == 0.0f) {
        // background keeps its input
        r[0] = *(const GMEM float*)((const GMEM char*)D.in_ao + (int64_t)y * D.in_ao_pitch + 4 * (int64_t)x);
        const GMEM float* gi = (const GMEM float*)((const GMEM char*)D.in_gi + (int64_t)y * D.in_gi_pitch) + 3 * (int64_t)x;
        const GMEM float* am = (const GMEM float*)((const GMEM char*)D.in_amb + (int64_t)y * D.in_amb_pitch) + 3 * (int64_t)x;
        r[1] = gi[0], r[2] = gi[1], r[3] = gi[2], r[4] = am[0], r[5] = am[1], r[6] = am[2];
    } else {
        const float4 Bp = sB[c];
        const float4 Cp = sC[c];
        const float zp = Ap.x, nx = Ap.y, ny = Ap.z, nz = Ap.w;
        // plane distance of a tap (a, b) cells away, scaled: with r(x, y) the pixel's view
        // ray, n_p . P_q = z_q (n_p . r_p + a nx S g / fx - b ny S g / fy), so
        // d = z_q t_ab - z_p t_00 with t linear in a and b
        const float sc = D.inv_sigma * kSqrtLog2e / zp;
        const float rx = ((float)x + 0.5f - D.cx) * D.inv_fx, ry = -((float)y + 0.5f - D.cy) * D.inv_fy;
        const float t0 = fmaf(nx, rx, fmaf(ny, ry, -nz)) * sc;
        const float tx = nx * (float)(S * D.g) * D.inv_fx * sc;
        const float ty = -ny * (float)(S * D.g) * D.inv_fy * sc;
        const float cps = zp * t0;
        constexpr float hc = (6.0f / 16) * (6.0f / 16);
        float sw = hc;
        float a0 = hc * Bp.x, a1 = hc * Bp.y, a2 = hc * Bp.z, a3 = hc * Bp.w, a4 = hc * Cp.x, a5 = hc * Cp.y,
              a6 = hc * Cp.z;
        // one row of five taps per iteration (unrolling all 24 taps would hoist every LDS
        // read and spill)
#pragma unroll 1
        for (int b = -2; b <= 2; ++b) {
            // log2 of the B3 weight of the row
            const float lhb = b == 0 ? -1.41503749927884382f : (b == 1 || b == -1) ? -2.0f : -4.0f;
            const int row = c + b * S * E;
            const float tb = fmaf((float)b, ty, t0);
#pragma unroll
            for (int a = -2; a <= 2; ++a) {
                if (a == 0 && b == 0) continue;
                const float lha = a == 0 ? -1.41503749927884382f : (a == 1 || a == -1) ? -2.0f : -4.0f;
                const int q = row + a * S;
                const float4 Aq = sA[q];
                const float d = fmaf(Aq.x, fmaf((float)a, tx, tb), -cps);
                const float cn = fmaxf(0.0f, fmaf(nx, Aq.y, fmaf(ny, Aq.z, nz * Aq.w)));
                // h_a h_b exp(-d^2) = 2^(log2 h_a + log2 h_b - (d sqrt(log2 e))^2)
                float w = __builtin_amdgcn_exp2f(fmaf(-d, d, lha + lhb)) * normal_weight<K2>(cn, D.normal_power);
                // off the image or on background: normal 0, so for k >= 1 the weight is
                // already 0; k = 0 needs the test
                if (K2 < 1) w = Aq.x > 0.0f ? w : 0.0f;
                const float4 Bq = sB[q];
                const float4 Cq = sC[q];
                sw += w;
                a0 = fmaf(w, Bq.x, a0);
                a1 = fmaf(w, Bq.y, a1);
                a2 = fmaf(w, Bq.z, a2);
                a3 = fmaf(w, Bq.w, a3);
                a4 = fmaf(w, Cq.x, a4);
                a5 = fmaf(w, Cq.y, a5);
                a6 = fmaf(w, Cq.z, a6);
            }
        }
        const float inv = __builtin_amdgcn_rcpf(sw);
        r[0] = a0 * inv, r[1] = a1 * inv, r[2] = a2 * inv, r[3] = a3 * inv, r[4] = a4 * inv, r[5] = a5 * inv,
        r[6] = a6 * inv;
    }
    *(GMEM float*)((GMEM char*)D.out_ao + (int64_t)y * D.out_ao_pitch + 4 * (int64_t)x) = r[0];
    GMEM float* go = (GMEM float*)((GMEM char*)D.out_gi + (int64_t)y * D.out_gi_pitch) + 3 * (int64_t)x;
    GMEM float* mo = (GMEM float*)((GMEM char*)D.out_amb + (int64_t)y * D.out_amb_pitch) + 3 * (int64_t)x;
    go[0] = r[1], go[1] = r[2], go[2] = r[3];
    mo[0] = r[4], mo[1] = r[5], mo[2] = r[6];
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
