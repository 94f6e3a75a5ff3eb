// gfx950 kernels of the visibility-bitmask gather.
//
// One thread owns one pixel and walks its N_d slices, both sides of each slice and N_s
// steps per side (Algorithm 1).  The hot loop per step: integer lattice -> depth gather
// -> slice-plane coordinates (c, h) of the sample -> front and back angles -> sector
// range -> newly covered sectors -> (rarely) normal + radiance gather for the indirect
// term -> OR into the slice mask.
//
// Numerics.  The slice frame (view vector, in-slice tangent, projected-normal angle) is
// built once per slice in FP64 and rounded to FP32; the per-sample angle-to-sector step
// runs in FP32.  A sector decision depends on which side of a boundary an endpoint
// falls.  When an FP32 endpoint lies within kGuard sectors of a boundary, that sample's
// decision is taken again in FP64 from the same FP32 inputs, so the kernel's masks are
// those of the FP64 definition unless an endpoint sits within FP64 rounding of a
// boundary.
#include <math.h>

#include <algorithm>

#include "ssvb_internal.h"

namespace ssvb {

constexpr float kInvPi32 = 10.185916357881302f;  // 32 / pi
constexpr double kInvPi32d = 10.185916357881301489;
constexpr double kPi = 3.141592653589793238;
constexpr float kGuard = 1.0f / 32768.0f;       // sectors; ~3e-6 rad
#ifndef SSVB_BATCH
#define SSVB_BATCH 4
#endif
#ifndef SSVB_WAVES
#define SSVB_WAVES 0
#endif
constexpr int kBatch = SSVB_BATCH;              // steps whose depth loads are issued together

// ---------------------------------------------------------------------------------------
// counter-based noise: PCG-RXS-M-XS hash (Jarzynski and Olano, JCGT 2020) and the R2
// dither of Roberts
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

__device__ __forceinline__ uint32_t pixel_hash(uint32_t x, uint32_t y, uint32_t s) {
    return pcg_hash(x + pcg_hash(y + pcg_hash(s)));
}

__device__ __forceinline__ uint32_t rotation16(const FrameArgs& A, int x, int y) {
    if (A.noise == SSVB_NOISE_FIXED) return 0u;
    if (A.noise == SSVB_NOISE_R2)
        return ((uint32_t)x * A.r2a1 + (uint32_t)y * A.r2a2 + A.seed * A.r2a3) >> 16;
    return pixel_hash((uint32_t)x, (uint32_t)y, A.seed) >> 16;
}

__device__ __forceinline__ uint32_t jitter8(const FrameArgs& A, int x, int y, int i) {
    if (A.noise == SSVB_NOISE_FIXED) return 0u;
    return pixel_hash((uint32_t)x, (uint32_t)y, A.seed + 1u + (uint32_t)i) >> 24;
}

// ---------------------------------------------------------------------------------------
// G-buffer access
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float depth_at(const FrameArgs& A, int x, int y) {
    const float* row = (const float*)((const char*)A.depth + (int64_t)y * A.depth_pitch);
    return row[x];
}

template <bool F16>
__device__ __forceinline__ float3 load3(const char* base, int64_t pitch, int ch, int x, int y) {
    const char* row = base + (int64_t)y * pitch;
    if (F16) {
        const _Float16* p = (const _Float16*)row + (int64_t)x * ch;
        return make_float3((float)p[0], (float)p[1], (float)p[2]);
    }
    const float* p = (const float*)row + (int64_t)x * ch;
    return make_float3(p[0], p[1], p[2]);
}

__device__ __forceinline__ bool is_geometry(float z) { return z > 0.0f && z < INFINITY; }

// bits [0, k) for 0 <= k <= 32
__device__ __forceinline__ uint32_t low_bits(int k) { return k >= 32 ? 0xFFFFFFFFu : ((1u << k) - 1u); }

// bits [a, b) of a 32-bit mask; empty when b <= a
__device__ __forceinline__ uint32_t range_bits(int a, int b) { return low_bits(b) & ~low_bits(a); }

// ---------------------------------------------------------------------------------------
// FP64 slice frame
// ---------------------------------------------------------------------------------------
struct Frame64 {
    double R, vx, vy, vz;      // |r_p| and v = -r_p / |r_p|
    double ex, ey, ez;         // unit in-slice tangent toward the slice direction
    double av, ae;             // D3 . v and D3 . e (D3: view direction of one LUT unit)
    double nv, ne, gamma;      // projected normal in (v, e) and its angle from v
};

__device__ __forceinline__ void pixel_ray64(const FrameArgs& A, int x, int y, Frame64& F) {
    const double rpx = ((double)x + 0.5 - (double)A.cx) / (double)A.fx;
    const double rpy = -((double)y + 0.5 - (double)A.cy) / (double)A.fy;
    F.R = sqrt(rpx * rpx + rpy * rpy + 1.0);
    F.vx = -rpx / F.R;
    F.vy = -rpy / F.R;
    F.vz = 1.0 / F.R;
}

__device__ __forceinline__ void slice_frame64(const FrameArgs& A, int Dx, int Dy, float3 n, Frame64& F) {
    const double d3x = (double)Dx / (4096.0 * (double)A.fx);
    const double d3y = -(double)Dy / (4096.0 * (double)A.fy);
    F.av = d3x * F.vx + d3y * F.vy;
    double ex = d3x - F.av * F.vx, ey = d3y - F.av * F.vy, ez = -F.av * F.vz;
    F.ae = sqrt(ex * ex + ey * ey + ez * ez);
    F.ex = ex / F.ae;
    F.ey = ey / F.ae;
    F.ez = ez / F.ae;
    F.nv = (double)n.x * F.vx + (double)n.y * F.vy + (double)n.z * F.vz;
    F.ne = (double)n.x * F.ex + (double)n.y * F.ey + (double)n.z * F.ez;
    F.gamma = (F.nv * F.nv + F.ne * F.ne < 1e-12) ? 0.0 : atan2(F.ne, F.nv);
}

// Sector range [a, b) of one sample decided in FP64 (used near a boundary).
template <int CRIT>
__device__ __noinline__ int2 decide64(const FrameArgs& A, int x, int y, float zp, float zs, int so,
                                      int Dx, int Dy, float3 n) {
    Frame64 F;
    pixel_ray64(A, x, y, F);
    slice_frame64(A, Dx, Dy, n, F);
    const double lam = (double)so / 16.0;
    const double zpd = zp, zsd = zs;
    const double tp = (double)A.t0 + (double)A.tk * zpd;
    const double c = -(zsd - zpd) * F.R + zsd * lam * F.av;
    const double h = fabs(zsd * lam * F.ae);
    const double sgn = so > 0 ? 1.0 : -1.0;
    double tf = sgn * atan2(h, c) - F.gamma;
    double tb = sgn * atan2(h, c - tp) - F.gamma;
    tf = fmin(fmax(tf, -0.5 * kPi), 0.5 * kPi);
    tb = fmin(fmax(tb, -0.5 * kPi), 0.5 * kPi);
    const double ulo = (fmin(tf, tb) + 0.5 * kPi) / kPi;
    const double uhi = (fmax(tf, tb) + 0.5 * kPi) / kPi;
    if (CRIT == SSVB_HIT_ROUND) {
        return make_int2((int)floor(32.0 * ulo + 0.5), (int)floor(32.0 * uhi + 0.5));
    } else {
        const int a = (int)floor(32.0 * ulo);
        const int w = (int)ceil(32.0 * (uhi - ulo));
        return make_int2(a, min(a + w, 32));
    }
}

__device__ __forceinline__ bool near_integer(float v) { return fabsf(v - rintf(v)) < kGuard; }

// atan2(y, x) for y > 0 and any x (including -inf), in (0, pi].  Octant reduction to
// r = min / max in [0, 1] and an odd minimax polynomial of degree 17 for atan(r) on
// [0, 1] (fitted offline; |error| < 1e-7 rad in FP32 evaluation).
__device__ __forceinline__ float atan2_pos(float y, float x) {
    const float ax = fabsf(x);
    const float mx = fmaxf(ax, y), mn = fminf(ax, y);
    const float r = mn * __builtin_amdgcn_rcpf(mx);
    const float r2 = r * r;
    float p = 0.0024567244108766317f;
    p = fmaf(p, r2, -0.014401358552277088f);
    p = fmaf(p, r2, 0.039781227707862854f);
    p = fmaf(p, r2, -0.07234857976436615f);
    p = fmaf(p, r2, 0.10498946905136108f);
    p = fmaf(p, r2, -0.14161229133605957f);
    p = fmaf(p, r2, 0.19985906779766083f);
    p = fmaf(p, r2, -0.33332598209381104f);
    p = fmaf(p, r2, 0.9999998807907104f);
    float a = p * r;
    if (y > ax) a = 1.57079632679489662f - a;
    if (x < 0.0f) a = 3.14159265358979324f - a;
    return a;
}

// ---------------------------------------------------------------------------------------
// the gather
// ---------------------------------------------------------------------------------------
enum { MODE_COMPUTE = 0, MODE_LATTICE = 1, MODE_ENDPOINTS = 2 };

__device__ __forceinline__ void store_background(const FrameArgs& A, int x, int y) {
    *(float*)((char*)A.ao + (int64_t)y * A.ao_pitch + (int64_t)x * 4) = 1.0f;
    float* g = (float*)((char*)A.gi + (int64_t)y * A.gi_pitch) + 3 * (int64_t)x;
    float* m = (float*)((char*)A.amb + (int64_t)y * A.amb_pitch) + 3 * (int64_t)x;
    g[0] = g[1] = g[2] = 0.0f;
    m[0] = m[1] = m[2] = 0.0f;
    if (A.masks) {
        uint32_t* mk = (uint32_t*)((char*)A.masks + (int64_t)y * A.masks_pitch) + (int64_t)x * A.nd;
        for (int i = 0; i < A.nd; ++i) mk[i] = 0u;
    }
}

// Per-slice constants of the hot loop (FP32, derived from the FP64 frame).
struct SliceF {
    float ex, ey, ez;   // unit tangent of the slice toward +d
    float nv, ne;       // centre normal in (v, e)
    float K;            // sector coordinate of the direction v: 16.5 - gamma * 32 / pi
    float avq, aeq;     // (D3 . v) / 16 and (D3 . e) / 16: per 1/16-px offset unit
    float cg, sg;       // unit projected normal (cos gamma, sin gamma)
};

__device__ __forceinline__ SliceF slice_constants(const FrameArgs& A, int x, int y, int2 D, float3 n) {
    Frame64 F;
    pixel_ray64(A, x, y, F);
    const double d3x = (double)D.x / (4096.0 * (double)A.fx);
    const double d3y = -(double)D.y / (4096.0 * (double)A.fy);
    const double av = d3x * F.vx + d3y * F.vy;
    const double ex = d3x - av * F.vx, ey = d3y - av * F.vy, ez = -av * F.vz;
    const double ae = sqrt(ex * ex + ey * ey + ez * ez);
    const double ie = 1.0 / ae;
    SliceF S;
    S.ex = (float)(ex * ie);
    S.ey = (float)(ey * ie);
    S.ez = (float)(ez * ie);
    const double nv = (double)n.x * F.vx + (double)n.y * F.vy + (double)n.z * F.vz;
    const double ne = ((double)n.x * ex + (double)n.y * ey + (double)n.z * ez) * ie;
    S.nv = (float)nv;
    S.ne = (float)ne;
    const double g2 = nv * nv + ne * ne;
    float gamma = 0.0f;
    S.cg = 1.0f;
    S.sg = 0.0f;
    if (g2 >= 1e-12) {
        const float gm = atan2_pos(fabsf(S.ne), S.nv);
        gamma = S.ne < 0.0f ? -gm : gm;
        const double ig = 1.0 / sqrt(g2);
        S.cg = (float)(nv * ig);
        S.sg = (float)(ne * ig);
    }
    S.K = fmaf(-gamma, kInvPi32, 16.5f);
    S.avq = (float)(av * 0.0625);
    S.aeq = (float)(ae * 0.0625);
    return S;
}

// 32-bit byte offset of texel (X, Y) in the depth image (the image spans < 4 GiB)
__device__ __forceinline__ uint32_t depth_off(const FrameArgs& A, int X, int Y) {
    return (uint32_t)Y * (uint32_t)A.depth_pitch + (uint32_t)X * 4u;
}

__device__ __forceinline__ float depth_load(const FrameArgs& A, uint32_t off) {
    return *(const float*)((const char*)A.depth + off);
}

// One sample of the march: sector range, newly covered sectors, indirect light.
template <int CRIT, bool EXACT, bool TINF, int FMT>
__device__ __forceinline__ void march_sample(const FrameArgs& A, const SliceF& S, int x, int y, float zp, float R,
                                             float vx, float vy, float vz, float tp, float3 n, int2 D, int s,
                                             int o, int X, int Y, bool ok, float zs, uint32_t& B, float& gir,
                                             float& gig, float& gib, bool& flagged) {
    ok = ok && is_geometry(zs);
    const float of = (float)o;
    const float sk = s > 0 ? kInvPi32 : -kInvPi32;
    // slice-plane coordinates of delta = s_f - p: c along v, h = |delta . e|
    const float c = fmaf(zs, of * (s > 0 ? S.avq : -S.avq), -R * (zs - zp));
    const float h = zs * (of * S.aeq);
    // front and back angles from v (the back sample lies t farther along -v)
    const float af = atan2_pos(h, c);
    const float ab = TINF ? 3.14159265358979324f : atan2_pos(h, c - tp);
    const float yf = fminf(fmaxf(fmaf(af, sk, S.K), 0.5f), 32.5f);
    const float yb = fminf(fmaxf(fmaf(ab, sk, S.K), 0.5f), 32.5f);
    const float lo = fminf(yf, yb), hi = fmaxf(yf, yb);
    int a, b;
    bool near;
    if (CRIT == SSVB_HIT_ROUND) {
        a = (int)floorf(lo);
        b = (int)floorf(hi);
        near = near_integer(lo) | near_integer(hi);
    } else {
        a = (int)floorf(lo - 0.5f);
        const float wf = hi - lo;
        b = min(a + (int)ceilf(wf), 32);
        near = near_integer(lo - 0.5f) | near_integer(wf);
    }
    near = near && ok;
    if (near) {
        if (EXACT) {
            const int2 ab64 = decide64<CRIT>(A, x, y, zp, zs, s * o, D.x, D.y, n);
            a = ab64.x;
            b = ab64.y;
        } else {
            flagged = true;
        }
    }
    const uint32_t m = ok ? range_bits(a, b) : 0u;
    const uint32_t fresh = m & ~B;
    if (fresh) {
        // indirect light from the newly covered sectors (Algorithm 1; Section 3.3)
        const float3 nj = load3<(FMT & 1) != 0>(A.normal, A.normal_pitch, A.normal_ch, X, Y);
        const float3 cj = load3<(FMT & 2) != 0>(A.radiance, A.radiance_pitch, A.radiance_ch, X, Y);
        const float hs = s > 0 ? h : -h;
        const float ndp = fmaf(S.nv, c, S.ne * hs);
        const float njv = nj.x * vx + nj.y * vy + nj.z * vz;
        const float nje = nj.x * S.ex + nj.y * S.ey + nj.z * S.ez;
        const float ndj = fmaf(njv, c, nje * hs);
        const float w =
            (float)__popc(fresh) * (1.0f / 32.0f) * fmaxf(ndp, 0.0f) * fmaxf(-ndj, 0.0f) / fmaf(c, c, h * h);
        gir = fmaf(w, cj.x, gir);
        gig = fmaf(w, cj.y, gig);
        gib = fmaf(w, cj.z, gib);
    }
    B |= m;
}

// One pixel of the gather.
//  CRIT   hit criterion
//  MODE   compute, or dump the lattice / the FP32 endpoint arguments (test hooks)
//  EXACT  false: FP32 decisions; a pixel with an endpoint within kGuard of a boundary
//         is appended to the fix-up list.  true: such samples are decided in FP64.
//  TINF   thickness is +inf: every back angle is pi, no second atan2
// Both sides of a slice advance together, one step per iteration: the + side only
// covers sectors at or above the direction v and the - side only sectors below it, so
// the two never compete for a sector and the interleaving leaves every mask, and
// every newly covered count, as a side-by-side march would produce it.
template <int CRIT, int MODE, bool EXACT, bool TINF, int FMT>
__device__ __forceinline__ void gather_pixel(const FrameArgs& A, int x, int y, int32_t* dbg_i, float* dbg_f) {
    const float zp = depth_at(A, x, y);
    const bool geom = is_geometry(zp);
    if (MODE == MODE_COMPUTE && !geom) {
        store_background(A, x, y);
        return;
    }
    const float3 n = MODE == MODE_LATTICE ? make_float3(0.0f, 0.0f, 1.0f)
                                          : load3<(FMT & 1) != 0>(A.normal, A.normal_pitch, A.normal_ch, x, y);
    const uint32_t rho = rotation16(A, x, y);

    // step length in 1/16 px: floor(C / z_p) from one IEEE FP32 division, clamped
    float quot = __fdiv_rn(A.c_step, geom ? zp : 1.0f);
    quot = fminf(quot, A.q_max_f);
    const int q = max((int)floorf(quot), A.q_min);
    const float tp = fmaf(A.tk, zp, A.t0);

    float R, vx, vy, vz;
    {
        Frame64 F;
        pixel_ray64(A, x, y, F);
        R = (float)F.R;
        vx = (float)F.vx;
        vy = (float)F.vy;
        vz = (float)F.vz;
    }

    float ao_acc = 0.0f;
    float gir = 0.0f, gig = 0.0f, gib = 0.0f;
    float amr = 0.0f, amg = 0.0f, amb = 0.0f;
    bool flagged = false;
    const int x16 = (x << 16) + 32768, y16 = (y << 16) + 32768;
    const uint32_t own = depth_off(A, x, y);

    for (int i = 0; i < A.nd; ++i) {
        const int k = (int)(((uint32_t)i * 65536u + rho) / (uint32_t)(16 * A.nd));
        const int2 D = A.lut[k];
        const int jit = (q * (int)jitter8(A, x, y, i)) >> 8;
        if (MODE == MODE_LATTICE) {
            for (int side = 0; side < 2; ++side) {
                const int s = side ? -1 : 1;
                for (int j = 0; j < A.ns; ++j) {
                    const int o = q * (j + 1) + jit;
                    int32_t* d = dbg_i + ((((int64_t)i * 2 + side) * A.ns + j) * 2);
                    d[0] = (x16 + s * o * D.x) >> 16;
                    d[1] = (y16 + s * o * D.y) >> 16;
                }
            }
            continue;
        }
        const SliceF S = slice_constants(A, x, y, D, n);
        uint32_t B = 0u;

        // steps are taken kBatch at a time: the depth loads of the whole batch (both
        // sides) are issued first, then the samples are consumed near to far
        for (int j0 = 0; j0 < A.ns; j0 += kBatch) {
            float zs[kBatch][2];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int o = q * (j0 + u + 1) + jit;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int so = side ? -o : o;
                    const int X = (x16 + so * D.x) >> 16, Y = (y16 + so * D.y) >> 16;
                    const bool ok = j0 + u < A.ns && (unsigned)X < (unsigned)A.W && (unsigned)Y < (unsigned)A.H &&
                                    !(X == x && Y == y) && geom;
                    zs[u][side] = depth_load(A, ok ? depth_off(A, X, Y) : own);
                }
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int j = j0 + u;
                if (j >= A.ns) break;
                const int o = q * (j + 1) + jit;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int s = side ? -1 : 1;
                    const int so = side ? -o : o;
                    const int X = (x16 + so * D.x) >> 16, Y = (y16 + so * D.y) >> 16;
                    const bool ok = (unsigned)X < (unsigned)A.W && (unsigned)Y < (unsigned)A.H && !(X == x && Y == y) &&
                                    geom;
                    if (MODE == MODE_ENDPOINTS) {
                        const float z = zs[u][side];
                        if (!(ok && is_geometry(z))) continue;
                        const float of = (float)o;
                        const float sk = side ? -kInvPi32 : kInvPi32;
                        const float c = fmaf(z, of * (side ? -S.avq : S.avq), -R * (z - zp));
                        const float h = z * (of * S.aeq);
                        const float af = atan2_pos(h, c);
                        const float ab = atan2_pos(h, c - tp);
                        const float yf = fminf(fmaxf(fmaf(af, sk, S.K), 0.5f), 32.5f);
                        const float yb = fminf(fmaxf(fmaf(ab, sk, S.K), 0.5f), 32.5f);
                        const float lo = fminf(yf, yb), hi = fmaxf(yf, yb);
                        float* d = dbg_f + ((((int64_t)i * 2 + side) * A.ns + j) * 2);
                        d[0] = CRIT == SSVB_HIT_ROUND ? lo : lo - 0.5f;
                        d[1] = CRIT == SSVB_HIT_ROUND ? hi : hi - lo;
                    } else {
                        march_sample<CRIT, EXACT, TINF, FMT>(A, S, x, y, zp, R, vx, vy, vz, tp, n, D, s, o, X, Y, ok,
                                                        zs[u][side], B, gir, gig, gib, flagged);
                    }
                }
            }
        }
        if (MODE != MODE_COMPUTE) continue;
        ao_acc += 1.0f - (float)__popc(B) * (1.0f / 32.0f);
        if (A.masks) {
            uint32_t* mk = (uint32_t*)((char*)A.masks + (int64_t)y * A.masks_pitch) + (int64_t)x * A.nd;
            mk[i] = B;
        }
        // directionally occluded ambient (Section 3.2)
        const int per = 32 / A.na;
        for (int kk = 0; kk < A.na; ++kk) {
            const uint32_t open = ~B & range_bits(kk * per, (kk + 1) * per);
            if (!open) continue;
            const float cps = S.cg * A.amb_cb[kk] - S.sg * A.amb_sb[kk];
            const float sps = S.sg * A.amb_cb[kk] + S.cg * A.amb_sb[kk];
            const float dvx = cps * vx + sps * S.ex, dvy = cps * vy + sps * S.ey, dvz = cps * vz + sps * S.ez;
            const float wx = A.Rvw[0] * dvx + A.Rvw[1] * dvy + A.Rvw[2] * dvz;
            const float wy = A.Rvw[3] * dvx + A.Rvw[4] * dvy + A.Rvw[5] * dvz;
            const float wz = A.Rvw[6] * dvx + A.Rvw[7] * dvy + A.Rvw[8] * dvz;
            // L2 real spherical harmonics
            const float b0 = 0.28209479177387814f;
            const float b1 = 0.48860251190291992f * wy, b2 = 0.48860251190291992f * wz,
                        b3 = 0.48860251190291992f * wx;
            const float b4 = 1.0925484305920792f * wx * wy, b5 = 1.0925484305920792f * wy * wz;
            const float b6 = 0.31539156525252005f * (3.0f * wz * wz - 1.0f);
            const float b7 = 1.0925484305920792f * wx * wz, b8 = 0.54627421529603959f * (wx * wx - wy * wy);
            const float* Sh = A.sh;
            const float Lr = b0 * Sh[0] + b1 * Sh[3] + b2 * Sh[6] + b3 * Sh[9] + b4 * Sh[12] + b5 * Sh[15] +
                             b6 * Sh[18] + b7 * Sh[21] + b8 * Sh[24];
            const float Lg = b0 * Sh[1] + b1 * Sh[4] + b2 * Sh[7] + b3 * Sh[10] + b4 * Sh[13] + b5 * Sh[16] +
                             b6 * Sh[19] + b7 * Sh[22] + b8 * Sh[25];
            const float Lb = b0 * Sh[2] + b1 * Sh[5] + b2 * Sh[8] + b3 * Sh[11] + b4 * Sh[14] + b5 * Sh[17] +
                             b6 * Sh[20] + b7 * Sh[23] + b8 * Sh[26];
            const float fr = (float)__popc(open) * (1.0f / 32.0f);
            amr = fmaf(fr, Lr, amr);
            amg = fmaf(fr, Lg, amg);
            amb = fmaf(fr, Lb, amb);
        }
    }
    if (MODE != MODE_COMPUTE) return;
    const float inv_nd = 1.0f / (float)A.nd;
    *(float*)((char*)A.ao + (int64_t)y * A.ao_pitch + (int64_t)x * 4) = ao_acc * inv_nd;
    float* g = (float*)((char*)A.gi + (int64_t)y * A.gi_pitch) + 3 * (int64_t)x;
    g[0] = gir * inv_nd;
    g[1] = gig * inv_nd;
    g[2] = gib * inv_nd;
    float* m = (float*)((char*)A.amb + (int64_t)y * A.amb_pitch) + 3 * (int64_t)x;
    m[0] = amr * inv_nd;
    m[1] = amg * inv_nd;
    m[2] = amb * inv_nd;
    if (!EXACT && flagged) {
        const uint32_t slot = atomicAdd(A.fix, 1u);
        A.fix[1 + slot] = (uint32_t)y * (uint32_t)A.W + (uint32_t)x;
    }
}

#if SSVB_WAVES > 0
#define SSVB_OCCUPANCY __attribute__((amdgpu_waves_per_eu(SSVB_WAVES, 8)))
#else
#define SSVB_OCCUPANCY
#endif

template <int CRIT, bool TINF, int FMT>
__global__ __launch_bounds__(256) SSVB_OCCUPANCY void gather_plain(FrameArgs A) {
    int tx, ty;
    if (!tile_of(A, blockIdx.x, tx, ty)) return;
    const int x = tx * A.tile_w + (int)(threadIdx.x % (unsigned)A.tile_w);
    const int y = ty * A.tile_h + (int)(threadIdx.x / (unsigned)A.tile_w);
    if (x >= A.W || y >= A.H) return;
    gather_pixel<CRIT, MODE_COMPUTE, false, TINF, FMT>(A, x, y, nullptr, nullptr);
}

// Re-run the pixels the main pass flagged, deciding near-boundary samples in FP64.
template <int CRIT, bool TINF, int FMT>
__global__ __launch_bounds__(64) void gather_fixup(FrameArgs A) {
    const uint32_t count = A.fix[0];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
        const uint32_t p = A.fix[1 + t];
        const int y = (int)(p / (uint32_t)A.W), x = (int)(p % (uint32_t)A.W);
        gather_pixel<CRIT, MODE_COMPUTE, true, TINF, FMT>(A, x, y, nullptr, nullptr);
    }
}

__global__ void reset_counter(uint32_t* c) { *c = 0u; }

__global__ __launch_bounds__(256) void debug_lattice(FrameArgs A, int32_t* out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= A.W || y >= A.H) return;
    int32_t* d = out + ((int64_t)y * A.W + x) * (int64_t)A.nd * 2 * A.ns * 2;
    gather_pixel<SSVB_HIT_ROUND, MODE_LATTICE, false, false, 0>(A, x, y, d, nullptr);
}

template <int CRIT, int FMT>
__global__ __launch_bounds__(256) void debug_endpoints(FrameArgs A, float* out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= A.W || y >= A.H) return;
    float* d = out + ((int64_t)y * A.W + x) * (int64_t)A.nd * 2 * A.ns * 2;
    gather_pixel<CRIT, MODE_ENDPOINTS, false, false, FMT>(A, x, y, nullptr, d);
}

// ---------------------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------------------
static dim3 plain_grid(const FrameArgs& A, dim3 block) {
    return dim3((A.W + block.x - 1) / block.x, (A.H + block.y - 1) / block.y);
}

template <int CRIT, bool TINF, int FMT>
static void launch_pair(const FrameArgs& A, hipStream_t stream) {
    const uint32_t nt = (uint32_t)A.tiles_x * A.tiles_y;
    const uint32_t nwg = A.xcd_remap ? kXcds * ((nt + kXcds - 1) / kXcds) : nt;
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, stream, A.fix);
    hipLaunchKernelGGL((gather_plain<CRIT, TINF, FMT>), dim3(nwg), dim3(A.tile_w * A.tile_h), 0, stream, A);
    const int64_t px = (int64_t)A.W * A.H;
    const int fix_blocks = (int)std::min<int64_t>(std::max<int64_t>((px / 64 + 15) / 16, 64), 4096);
    hipLaunchKernelGGL((gather_fixup<CRIT, TINF, FMT>), dim3(fix_blocks), dim3(64), 0, stream, A);
}

template <int CRIT, bool TINF>
static void launch_fmt(const FrameArgs& A, hipStream_t stream) {
    switch (A.normal_f16 | (A.radiance_f16 << 1)) {
        case 0: launch_pair<CRIT, TINF, 0>(A, stream); break;
        case 1: launch_pair<CRIT, TINF, 1>(A, stream); break;
        case 2: launch_pair<CRIT, TINF, 2>(A, stream); break;
        default: launch_pair<CRIT, TINF, 3>(A, stream); break;
    }
}

hipError_t launch_plain(const FrameArgs& A, hipStream_t stream) {
    const bool tinf = isinf(A.t0);
    if (A.criterion == SSVB_HIT_ROUND) {
        if (tinf) launch_fmt<SSVB_HIT_ROUND, true>(A, stream);
        else launch_fmt<SSVB_HIT_ROUND, false>(A, stream);
    } else {
        if (tinf) launch_fmt<SSVB_HIT_PSEUDOCODE, true>(A, stream);
        else launch_fmt<SSVB_HIT_PSEUDOCODE, false>(A, stream);
    }
    return hipGetLastError();
}

hipError_t launch_debug_lattice(const FrameArgs& A, int32_t* out, hipStream_t stream) {
    const dim3 block(16, 16);
    hipLaunchKernelGGL(debug_lattice, plain_grid(A, block), block, 0, stream, A, out);
    return hipGetLastError();
}

template <int CRIT>
static void launch_endpoints_fmt(const FrameArgs& A, float* out, hipStream_t stream) {
    const dim3 block(16, 16);
    switch (A.normal_f16) {
        case 0: hipLaunchKernelGGL((debug_endpoints<CRIT, 0>), plain_grid(A, block), block, 0, stream, A, out); break;
        default: hipLaunchKernelGGL((debug_endpoints<CRIT, 1>), plain_grid(A, block), block, 0, stream, A, out); break;
    }
}

hipError_t launch_debug_endpoints(const FrameArgs& A, float* out, hipStream_t stream) {
    if (A.criterion == SSVB_HIT_ROUND) launch_endpoints_fmt<SSVB_HIT_ROUND>(A, out, stream);
    else launch_endpoints_fmt<SSVB_HIT_PSEUDOCODE>(A, out, stream);
    return hipGetLastError();
}

}  // namespace ssvb
