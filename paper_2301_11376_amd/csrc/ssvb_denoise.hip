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
// so every tap is an LDS read; the pass is ALU-bound (about 30 VALU operations per tap).
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

template <int S>
__global__ __launch_bounds__(kThreads) void denoise_pass(DenoiseArgs D) {
    constexpr int E = kDenoiseTile + 4 * S;  // staged tile edge, cells
    constexpr int N = E * E;
    __shared__ float4 sP[N];  // position xyz, 1 on foreground (0 elsewhere)
    __shared__ float4 sN[N];  // unit normal xyz, AO
    __shared__ float4 sG[N];  // GI rgb, ambient r
    __shared__ float2 sA[N];  // ambient g b
    const int tile = (int)blockIdx.x;
    const int u0 = (tile % D.tiles_x) * kDenoiseTile - 2 * S;
    const int v0 = (tile / D.tiles_x) * kDenoiseTile - 2 * S;

    for (int i = (int)threadIdx.x; i < N; i += kThreads) {
        const int u = u0 + i % E, v = v0 + i / E;
        float4 P = make_float4(0.0f, 0.0f, 0.0f, 0.0f), Nn = P, G = P;
        float2 Am = make_float2(0.0f, 0.0f);
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
                const float il = l2 > 0.0f ? 1.0f / sqrtf(l2) : 0.0f;
                P = make_float4(z * (((float)x + 0.5f - D.cx) * D.inv_fx), -z * (((float)y + 0.5f - D.cy) * D.inv_fy), -z,
                                1.0f);
                const float ao = *(const GMEM float*)((const GMEM char*)D.in_ao + (int64_t)y * D.in_ao_pitch + 4 * (int64_t)x);
                Nn = make_float4(nx * il, ny * il, nz * il, ao);
                const GMEM float* gi = (const GMEM float*)((const GMEM char*)D.in_gi + (int64_t)y * D.in_gi_pitch) + 3 * (int64_t)x;
                const GMEM float* am = (const GMEM float*)((const GMEM char*)D.in_amb + (int64_t)y * D.in_amb_pitch) + 3 * (int64_t)x;
                G = make_float4(gi[0], gi[1], gi[2], am[0]);
                Am = make_float2(am[1], am[2]);
            }
        }
        sP[i] = P;
        sN[i] = Nn;
        sG[i] = G;
        sA[i] = Am;
    }
    __syncthreads();

    const int lx = (int)threadIdx.x % kDenoiseTile, ly = (int)threadIdx.x / kDenoiseTile;
    const int u = u0 + 2 * S + lx, v = v0 + 2 * S + ly;
    if (u >= D.gw || v >= D.gh) return;
    const int x = u * D.g, y = v * D.g;
    const int c = (ly + 2 * S) * E + lx + 2 * S;
    const float4 Pp = sP[c];
    float r[7];
    if (Pp.w == 0.0f) {
        // background keeps its input
        r[0] = *(const GMEM float*)((const GMEM char*)D.in_ao + (int64_t)y * D.in_ao_pitch + 4 * (int64_t)x);
        const GMEM float* gi = (const GMEM float*)((const GMEM char*)D.in_gi + (int64_t)y * D.in_gi_pitch) + 3 * (int64_t)x;
        const GMEM float* am = (const GMEM float*)((const GMEM char*)D.in_amb + (int64_t)y * D.in_amb_pitch) + 3 * (int64_t)x;
        r[1] = gi[0], r[2] = gi[1], r[3] = gi[2], r[4] = am[0], r[5] = am[1], r[6] = am[2];
    } else {
        const float4 Np = sN[c];
        const float4 Gp = sG[c];
        const float2 Ap = sA[c];
        constexpr float hc = (6.0f / 16) * (6.0f / 16);
        const float cp = fmaf(Np.x, Pp.x, fmaf(Np.y, Pp.y, Np.z * Pp.z));  // n_p . P_p
        const float sc = D.inv_sigma / -Pp.z;                               // 1 / (sigma z_p)
        float sw = hc;
        float a0 = hc * Np.w, a1 = hc * Gp.x, a2 = hc * Gp.y, a3 = hc * Gp.z, a4 = hc * Gp.w, a5 = hc * Ap.x,
              a6 = hc * Ap.y;
        // one row of five taps per iteration (unrolling all 24 taps would hoist every LDS
        // read and spill)
#pragma unroll 1
        for (int b = -2; b <= 2; ++b) {
            const float hb = b == 0 ? 6.0f / 16 : (b == 1 || b == -1) ? 4.0f / 16 : 1.0f / 16;
            const int row = c + b * S * E;
#pragma unroll
            for (int a = -2; a <= 2; ++a) {
                if (a == 0 && b == 0) continue;
                const float ha = a == 0 ? 6.0f / 16 : (a == 1 || a == -1) ? 4.0f / 16 : 1.0f / 16;
                const int q = row + a * S;
                const float4 Pq = sP[q];
                const float4 Nq = sN[q];
                const float d = (fmaf(Np.x, Pq.x, fmaf(Np.y, Pq.y, Np.z * Pq.z)) - cp) * sc;
                const float cn = fmaxf(0.0f, fmaf(Np.x, Nq.x, fmaf(Np.y, Nq.y, Np.z * Nq.z)));
                const float w = (ha * hb) * Pq.w * __expf(-d * d) * ipow(cn, D.normal_power);
                const float4 Gq = sG[q];
                const float2 Aq = sA[q];
                sw += w;
                a0 = fmaf(w, Nq.w, a0);
                a1 = fmaf(w, Gq.x, a1);
                a2 = fmaf(w, Gq.y, a2);
                a3 = fmaf(w, Gq.z, a3);
                a4 = fmaf(w, Gq.w, a4);
                a5 = fmaf(w, Aq.x, a5);
                a6 = fmaf(w, Aq.y, a6);
            }
        }
        r[0] = a0 / sw, r[1] = a1 / sw, r[2] = a2 / sw, r[3] = a3 / sw, r[4] = a4 / sw, r[5] = a5 / sw,
        r[6] = a6 / sw;
    }
    *(GMEM float*)((GMEM char*)D.out_ao + (int64_t)y * D.out_ao_pitch + 4 * (int64_t)x) = r[0];
    GMEM float* go = (GMEM float*)((GMEM char*)D.out_gi + (int64_t)y * D.out_gi_pitch) + 3 * (int64_t)x;
    GMEM float* mo = (GMEM float*)((GMEM char*)D.out_amb + (int64_t)y * D.out_amb_pitch) + 3 * (int64_t)x;
    go[0] = r[1], go[1] = r[2], go[2] = r[3];
    mo[0] = r[4], mo[1] = r[5], mo[2] = r[6];
}

}  // namespace

hipError_t launch_denoise(const DenoiseArgs& D, int pass, hipStream_t stream) {
    if (D.tiles <= 0) return hipSuccess;
    switch (pass) {
        case 0: hipLaunchKernelGGL(denoise_pass<1>, dim3(D.tiles), dim3(kThreads), 0, stream, D); break;
        case 1: hipLaunchKernelGGL(denoise_pass<2>, dim3(D.tiles), dim3(kThreads), 0, stream, D); break;
        case 2: hipLaunchKernelGGL(denoise_pass<4>, dim3(D.tiles), dim3(kThreads), 0, stream, D); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ssvb
