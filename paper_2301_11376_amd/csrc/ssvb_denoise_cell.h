// The denoiser's per-cell code: staging one cell of a tile's apron and filtering one output
// cell over its 5 x 5 taps (the a-trous pass of ssvb_denoise.hip).  The functions are
// __host__ __device__: the kernel calls them on its LDS arrays, and a test build runs them
// on the CPU.  The device primitives (reciprocal square root, exp2, reciprocal) have host
// forms here for that build only.
#ifndef SSVB_DENOISE_CELL_H
#define SSVB_DENOISE_CELL_H

#include <hip/hip_runtime.h>
#include <math.h>

#include "ssvb_denoise.h"

#ifdef __HIP_DEVICE_COMPILE__
#define DGMEM __attribute__((address_space(1)))
#else
#define DGMEM
#endif
#define SSVB_DHD __host__ __device__ __forceinline__

namespace ssvb {
namespace dn {

SSVB_DHD bool foreground(float z) { return z > 0.0f && z < INFINITY; }

SSVB_DHD float ipow(float c, int k) {
    float r = 1.0f;
    for (int e = k; e != 0; e >>= 1) {
        if (e & 1) r *= c;
        c *= c;
    }
    return r;
}

// c^k: K2 >= 0 means k = 2^K2 (K2 squarings), else the general square-and-multiply
template <int K2>
SSVB_DHD float normal_weight(float c, int k) {
    if (K2 < 0) return ipow(c, k);
#pragma unroll
    for (int i = 0; i < (K2 < 0 ? 0 : K2); ++i) c *= c;
    return c;
}

// hardware approximations on the device (about 1 ulp); exact forms on the host
SSVB_DHD float rsq(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}
SSVB_DHD float exp2_(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_exp2f(x);
#else
    return exp2f(x);
#endif
}
SSVB_DHD float rcp(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

constexpr float kSqrtLog2e = 1.20112240878644980f;  // sqrt(log2(e)): exp(-d^2) = 2^-(d sqrt(log2 e))^2

// Cell (u, v) as staged, for a cell inside the grid (0 <= u < gw, 0 <= v < gh; the
// caller leaves cells outside at zero): A = (depth, unit normal), B = (AO, GI rgb),
// C = (ambient rgb, 0); A, B and C are left as they are (zero) on background.
SSVB_DHD void stage_cell(const DenoiseArgs& D, int u, int v, float4& A, float4& B, float4& C) {
    const int x = u * D.g, y = v * D.g;
    const float z = *(const DGMEM float*)((const DGMEM char*)D.depth + (int64_t)y * D.depth_pitch + 4 * (int64_t)x);
    if (foreground(z)) {
        const DGMEM char* nb = (const DGMEM char*)D.normal + (int64_t)y * D.normal_pitch;
        float nx, ny, nz;
        if (D.normal_f16) {
            const DGMEM _Float16* p = (const DGMEM _Float16*)nb + (int64_t)x * D.normal_ch;
            nx = (float)p[0], ny = (float)p[1], nz = (float)p[2];
        } else {
            const DGMEM float* p = (const DGMEM float*)nb + (int64_t)x * D.normal_ch;
            nx = p[0], ny = p[1], nz = p[2];
        }
        const float l2 = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
        const float il = l2 > 0.0f ? rsq(l2) : 0.0f;
        A = make_float4(z, nx * il, ny * il, nz * il);
        const DGMEM float* gi = (const DGMEM float*)((const DGMEM char*)D.in_gi + (int64_t)y * D.in_gi_pitch) + 3 * (int64_t)x;
        const DGMEM float* am = (const DGMEM float*)((const DGMEM char*)D.in_amb + (int64_t)y * D.in_amb_pitch) + 3 * (int64_t)x;
        B = make_float4(*(const DGMEM float*)((const DGMEM char*)D.in_ao + (int64_t)y * D.in_ao_pitch + 4 * (int64_t)x),
                        gi[0], gi[1], gi[2]);
        C = make_float4(am[0], am[1], am[2], 0.0f);
    }
}

// Output cell (lx, ly) of the 16 x 16-cell tile whose staged block (edge E = 16 + 4 S
// cells, row-major in sA / sB / sC) starts at cell (u0, v0): the weighted average over
// the 5 x 5 taps S cells apart, or the input for a background cell; written to the
// outputs.  Cells outside the grid are skipped.
template <int S, int K2>
SSVB_DHD void filter_cell(const DenoiseArgs& D, const float4* sA, const float4* sB, const float4* sC, int u0, int v0,
                          int lx, int ly) {
    constexpr int E = kDenoiseTile + 4 * S;
    const int u = u0 + 2 * S + lx, v = v0 + 2 * S + ly;
    if (u >= D.gw || v >= D.gh) return;
    const int x = u * D.g, y = v * D.g;
    const int c = (ly + 2 * S) * E + lx + 2 * S;
    const float4 Ap = sA[c];
    float r[7];
    if (Ap.x == 0.0f) {
        // background keeps its input
        r[0] = *(const DGMEM float*)((const DGMEM char*)D.in_ao + (int64_t)y * D.in_ao_pitch + 4 * (int64_t)x);
        const DGMEM float* gi = (const DGMEM float*)((const DGMEM char*)D.in_gi + (int64_t)y * D.in_gi_pitch) + 3 * (int64_t)x;
        const DGMEM float* am = (const DGMEM float*)((const DGMEM char*)D.in_amb + (int64_t)y * D.in_amb_pitch) + 3 * (int64_t)x;
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
                float w = exp2_(fmaf(-d, d, lha + lhb)) * normal_weight<K2>(cn, D.normal_power);
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
        const float inv = rcp(sw);
        r[0] = a0 * inv, r[1] = a1 * inv, r[2] = a2 * inv, r[3] = a3 * inv, r[4] = a4 * inv, r[5] = a5 * inv,
        r[6] = a6 * inv;
    }
    *(DGMEM float*)((DGMEM char*)D.out_ao + (int64_t)y * D.out_ao_pitch + 4 * (int64_t)x) = r[0];
    DGMEM float* go = (DGMEM float*)((DGMEM char*)D.out_gi + (int64_t)y * D.out_gi_pitch) + 3 * (int64_t)x;
    DGMEM float* mo = (DGMEM float*)((DGMEM char*)D.out_amb + (int64_t)y * D.out_amb_pitch) + 3 * (int64_t)x;
    go[0] = r[1], go[1] = r[2], go[2] = r[3];
    mo[0] = r[4], mo[1] = r[5], mo[2] = r[6];
}

}  // namespace dn
}  // namespace ssvb

#endif
