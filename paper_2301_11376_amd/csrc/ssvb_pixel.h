// The per-pixel code of the visibility-bitmask gather (Algorithm 1 with the ambient split
// of Section 3.2), called by the gfx950 kernels in ssvb_kernels.hip.
//
// One thread owns one pixel and walks its N_d slices; each step advances both sides of
// the slice (Algorithm 1).  Per step and side: integer lattice -> depth gather ->
// slice-plane coordinates (c, h) of the sample -> front and back angles -> sector range
// -> newly covered sectors -> (when there are any) normal + radiance gather for the
// indirect term -> OR into the slice mask.
//
// Numerics.  The slice frame (view vector, in-slice tangent, projected normal) is built
// once per slice in FP64 and rounded to FP32; the per-sample angle-to-sector step runs in
// FP32.  A sector decision only depends on which side of a boundary direction an
// endpoint lies.  When an FP32 endpoint is within kGuard sectors of a boundary, the
// kernel decides it exactly: in FP64, from the same FP32 inputs, as the sign of the cross
// product between the sample direction and the boundary direction (boundary angles are
// multiples of pi/64 from the projected normal, whose cosine and sine come from a table
// and from the normal itself, so no transcendental function is evaluated).  The masks
// are therefore those of the FP64 definition unless an endpoint sits within FP64
// rounding of a boundary.
//
// Every function here is __host__ __device__.  The library calls them from its kernels
// only; the host forms of the few device primitives below exist for the CPU test build
// of this header, which runs the same per-pixel code on the host against the FP64
// oracle.
#pragma once

#include <math.h>

#include <algorithm>

#include "ssvb_internal.h"

namespace ssvb {

constexpr float kInvPi = 0.318309886183790672f;   // 1 / pi; N_b / pi = N_b * kInvPi exactly (N_b = 2^k)
constexpr float kGuard = 1.0f / 32768.0f;       // sectors at N_b = 32 (~3e-6 rad); scaled by N_b / 32
#ifndef SSVB_BATCH
#define SSVB_BATCH 1
#endif
constexpr int kBatch = SSVB_BATCH;              // steps whose depth loads are issued together
constexpr int kBlock = 256;                     // threads per workgroup

// ---------------------------------------------------------------------------------------
// device primitives (and their host forms for the CPU test build)
// ---------------------------------------------------------------------------------------
// Images and outputs live in global device memory.  Pointers read from a descriptor in
// memory are generic to the compiler; accessing them through pointers of the global
// address space lets it use global (rather than flat) loads and stores.
#if defined(__HIP_DEVICE_COMPILE__)
#define GMEM __attribute__((address_space(1)))
#else
#define GMEM
#endif

// 1 / x to about 1 ulp (the hardware reciprocal; exact division on the host)
SSVB_HD float rcp_approx(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// a / b correctly rounded (IEEE FP32 division)
SSVB_HD float div_rn(float a, float b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __fdiv_rn(a, b);
#else
    return a / b;
#endif
}

SSVB_HD int popc32(uint32_t v) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __popc(v);
#else
    return __builtin_popcount(v);
#endif
}

// v of the lane whose index differs in the bits of `mask` (the host build runs one lane
// per pixel, where no exchange happens)
SSVB_HD float lane_xor(float v, int mask) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __shfl_xor(v, mask);
#else
    (void)mask;
    return v;
#endif
}

// this thread's slot in the workgroup's LDS arrays (one slot on the host)
SSVB_HD int thread_index() {
#if defined(__HIP_DEVICE_COMPILE__)
    return (int)threadIdx.x;
#else
    return 0;
#endif
}

// ---------------------------------------------------------------------------------------
// counter-based noise: PCG-RXS-M-XS hash (Jarzynski and Olano, JCGT 2020) and the R2
// dither of Roberts
// ---------------------------------------------------------------------------------------
SSVB_HD uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

SSVB_HD uint32_t pixel_hash(uint32_t x, uint32_t y, uint32_t s) {
    return pcg_hash(x + pcg_hash(y + pcg_hash(s)));
}

SSVB_HD uint32_t rotation16(const FrameArgs& A, int x, int y) {
    if (A.noise == SSVB_NOISE_FIXED) return 0u;
    if (A.noise == SSVB_NOISE_R2)
        return ((uint32_t)x * A.r2a1 + (uint32_t)y * A.r2a2 + A.seed * A.r2a3) >> 16;
    return pixel_hash((uint32_t)x, (uint32_t)y, A.seed) >> 16;
}

SSVB_HD uint32_t jitter8(const FrameArgs& A, int x, int y, int i) {
    if (A.noise == SSVB_NOISE_FIXED) return 0u;
    return pixel_hash((uint32_t)x, (uint32_t)y, A.seed + 1u + (uint32_t)i) >> 24;
}

// ---------------------------------------------------------------------------------------
// G-buffer access (every image spans less than 4 GiB: 32-bit byte offsets)
// ---------------------------------------------------------------------------------------

#if !defined(__HIP_DEVICE_COMPILE__)
// Host build only: an observer of every image read (address, bytes), for the CPU cache
// model of the reads; null unless a test sets it.
inline void (*host_read_observer)(const void* addr, int bytes) = nullptr;
#define SSVB_OBSERVE_READ(p, n) \
    do {                        \
        if (host_read_observer) host_read_observer((p), (n)); \
    } while (0)
#else
#define SSVB_OBSERVE_READ(p, n) \
    do {                        \
    } while (0)
#endif

SSVB_HD float depth_load(const FrameArgs& A, uint32_t off) {
    SSVB_OBSERVE_READ((const char*)A.depth + off, 4);
    return *(const GMEM float*)((const GMEM char*)A.depth + off);
}

// F: 0 = FP32, 1 = FP16, -1 = given at run time by `f16`
template <int F>
SSVB_HD float3 load3(const char* base, int64_t pitch, int ch, int f16, int x, int y) {
    const bool h = F < 0 ? f16 != 0 : F == 1;
    const GMEM char* b = (const GMEM char*)base + image_off(pitch, ch, h, x, y);
    SSVB_OBSERVE_READ((const char*)b, h ? 6 : 12);
    if (h) {
        const GMEM _Float16* p = (const GMEM _Float16*)b;
        return make_float3((float)p[0], (float)p[1], (float)p[2]);
    }
    const GMEM float* p = (const GMEM float*)b;
    return make_float3(p[0], p[1], p[2]);
}

SSVB_HD bool is_geometry(float z) { return z > 0.0f && z < INFINITY; }

// bits [0, k) for 0 <= k <= 32 (the 64-bit shift makes k = 32 need no special case)
SSVB_HD uint32_t low_bits(int k) { return (uint32_t)(1ull << k) - 1u; }

// bits [a, b) of a 32-bit mask, for 0 <= a <= b <= 32 (every caller orders its ends)
SSVB_HD uint32_t range_bits(int a, int b) { return low_bits(b) - low_bits(a); }

// Within the guard band of an integer sector coordinate (the FP32 error in sectors grows
// with N_b, so the band does too).
template <int NB>
SSVB_HD bool near_integer(float v) { return fabsf(v - rintf(v)) < kGuard * (NB / 32); }

// Visibility mask of one slice: N_b sectors in N_b / 32 words, sector k in bit k % 32 of
// word k / 32.  Above 32 sectors a slice's mask also carries its number of set sectors,
// kept up to date by cover().
template <int NB>
struct SMask {
    static constexpr int W = NB / 32;
    uint32_t w[W];
    int n;
};

template <int NB>
SSVB_HD SMask<NB> mask_none() {
    SMask<NB> m;
#pragma unroll
    for (int i = 0; i < SMask<NB>::W; ++i) m.w[i] = 0u;
    m.n = 0;
    return m;
}

// Word I of 2^c mod 2^128, for c clamped to word I's span [32 I, 32 I + 32]: that is
// 2^(c - 32 I) mod 2^32.  The 64-bit shift reads its amount mod 64, so the low half of
// 2^(c mod 64) is word I for even I and the high half is word I for odd I (c = 32 I + 32
// of an odd word wraps to 2^0, whose high half is 0, as it should be).
template <int I>
SSVB_HD uint32_t pow2_word(int c) {
    c = min(max(c, 32 * I), 32 * I + 32);
    const uint64_t p = 1ull << (c & 63);
    return (I & 1) ? (uint32_t)(p >> 32) : (uint32_t)p;
}

template <int NB, int I = 0>
SSVB_HD void range_words(SMask<NB>& m, int a, int b) {
    if constexpr (I < SMask<NB>::W) {
        // bits [a, b) of word I: 2^b - 2^a in that word, mod 2^32
        m.w[I] = pow2_word<I>(b) - pow2_word<I>(a);
        range_words<NB, I + 1>(m, a, b);
    }
}

// sectors [a, b) for 0 <= a <= b <= N_b
template <int NB>
SSVB_HD SMask<NB> mask_range(int a, int b) {
    SMask<NB> m;
    if constexpr (NB == 32) {
        m.w[0] = range_bits(a, b);
    } else {
        range_words<NB>(m, a, b);
    }
    m.n = 0;
    return m;
}

// B |= m; returns the number of sectors of m not already in B.  Above 32 sectors this is
// the change in B's count (one popcount pass over the updated words, no m & ~B pass).
template <int NB>
SSVB_HD int cover(SMask<NB>& B, const SMask<NB>& m) {
    if constexpr (NB == 32) {
        const int c = popc32(m.w[0] & ~B.w[0]);
        B.w[0] |= m.w[0];
        return c;
    } else {
        int n = 0;
#pragma unroll
        for (int i = 0; i < SMask<NB>::W; ++i) {
            B.w[i] |= m.w[i];
            n += popc32(B.w[i]);
        }
        const int c = n - B.n;
        B.n = n;
        return c;
    }
}

// m & ~B
template <int NB>
SSVB_HD SMask<NB> mask_and_not(const SMask<NB>& m, const SMask<NB>& B) {
    SMask<NB> r;
#pragma unroll
    for (int i = 0; i < SMask<NB>::W; ++i) r.w[i] = m.w[i] & ~B.w[i];
    return r;
}

template <int NB>
SSVB_HD int mask_popc(const SMask<NB>& m) {
    int c = 0;
#pragma unroll
    for (int i = 0; i < SMask<NB>::W; ++i) c += popc32(m.w[i]);
    return c;
}

template <int NB>
SSVB_HD bool mask_any(const SMask<NB>& m) {
    uint32_t o = 0u;
#pragma unroll
    for (int i = 0; i < SMask<NB>::W; ++i) o |= m.w[i];
    return o != 0u;
}

// atan2(y, x) for y >= 0 and any x (including -inf), in [0, pi].  Octant reduction to
// r = min / max in [0, 1] and an odd minimax polynomial of degree 13 for atan(r) on
// [0, 1] (fitted offline; |error| < 3.3e-7 rad in FP32 evaluation on exact arguments,
// < 5.5e-7 rad with the rounding of r and of the reflections pi/2 - a and pi - a).
SSVB_HD float atan2_pos(float y, float x) {
    const float ax = fabsf(x);
    const float mx = fmaxf(ax, y), mn = fminf(ax, y);
    const float r = mn * rcp_approx(mx);
    const float r2 = r * r;
    float p = 0.006811789236962795f;
    p = fmaf(p, r2, -0.0336042121052742f);
    p = fmaf(p, r2, 0.07962366938591003f);
    p = fmaf(p, r2, -0.1323334276676178f);
    p = fmaf(p, r2, 0.19807815551757812f);
    p = fmaf(p, r2, -0.3331736922264099f);
    p = fmaf(p, r2, 0.9999961256980896f);
    float a = p * r;
    if (y > ax) a = 1.57079632679489662f - a;
    if (x < 0.0f) a = 3.14159265358979324f - a;
    return a;
}

// ---------------------------------------------------------------------------------------
// slice frame
// ---------------------------------------------------------------------------------------
// Per-slice constants of the hot loop (FP32, rounded from FP64).
struct SliceF {
    float ex, ey, ez;   // unit tangent of the slice toward +d
    float nv, ne;       // centre normal in (v, e)
    float K;            // sector coordinate of the direction v: N_b / 2 + 1/2 - gamma N_b / pi
    float avq, aeq;     // (D3 . v) / 16 and (D3 . e) / 16: per 1/16-px offset unit
    float cg, sg;       // unit projected normal (cos gamma, sin gamma)
};

// FP64 constants the exact decision needs, one slot per thread in LDS (struct of arrays)
struct ExactLds {
    double R[kBlock], tp[kBlock], av[kBlock], ae[kBlock], cg[kBlock], sg[kBlock];
};

template <int NB>
SSVB_HD SliceF slice_constants(const FrameArgs& A, double rpx, double rpy, int2 D, float3 n,
                                                  ExactLds& L, int t) {
    const double R = sqrt(rpx * rpx + rpy * rpy + 1.0);
    const double vx = -rpx / R, vy = -rpy / R, vz = 1.0 / R;
    const double d3x = (double)D.x / (4096.0 * (double)A.fx);
    const double d3y = -(double)D.y / (4096.0 * (double)A.fy);
    const double av = d3x * vx + d3y * vy;
    const double ex = d3x - av * vx, ey = d3y - av * vy, ez = -av * vz;
    const double ae = sqrt(ex * ex + ey * ey + ez * ez);
    const double ie = 1.0 / ae;
    SliceF S;
    S.ex = (float)(ex * ie);
    S.ey = (float)(ey * ie);
    S.ez = (float)(ez * ie);
    const double nv = (double)n.x * vx + (double)n.y * vy + (double)n.z * vz;
    const double ne = ((double)n.x * ex + (double)n.y * ey + (double)n.z * ez) * ie;
    S.nv = (float)nv;
    S.ne = (float)ne;
    const double g2 = nv * nv + ne * ne;
    float gamma = 0.0f;
    double cg = 1.0, sg = 0.0;
    if (g2 >= 1e-12) {
        const float gm = atan2_pos(fabsf(S.ne), S.nv);
        gamma = S.ne < 0.0f ? -gm : gm;
        const double ig = 1.0 / sqrt(g2);
        cg = nv * ig;
        sg = ne * ig;
    }
    S.cg = (float)cg;
    S.sg = (float)sg;
    S.K = fmaf(-gamma, (float)NB * kInvPi, (float)(NB / 2) + 0.5f);
    S.avq = (float)(av * 0.0625);
    S.aeq = (float)(ae * 0.0625);
    L.av[t] = av;
    L.ae[t] = ae;
    L.cg[t] = cg;
    L.sg[t] = sg;
    return S;
}

// ---------------------------------------------------------------------------------------
// exact decisions near a sector boundary
// ---------------------------------------------------------------------------------------
// Is the direction (sv, se) (in the slice, from v toward e) at or counter-clockwise of
// the direction at angle h pi / (2 N_b) from the projected normal (cg, sg)?
// Products are rounded separately (no contraction), so a cross product of two identical
// directions is exactly zero.
template <int NB>
SSVB_HD bool at_or_above(const FrameArgs& A, int h, double cg, double sg, double sv, double se) {
#pragma clang fp contract(off)
    // cos, sin of h pi / (2 N_b), h = -2 N_b .. 2 N_b
    const GMEM double* hs = (const GMEM double*)A.half_sector + 2 * (h + 2 * NB);
    const double2 cs = make_double2(hs[0], hs[1]);
    const double dv = cs.x * cg - cs.y * sg, de = cs.y * cg + cs.x * sg;
    return dv * se - de * sv >= 0.0;
}

// Exact floor of the FP32 sector coordinate `y` (ROUND: y = N_b u + 1/2; PSEUDOCODE:
// y = N_b u) of an endpoint with direction (sv, se), given that y is near the integer m.
// The angle is clamped to the hemisphere first, so the floor never drops below 0.
template <int NB>
SSVB_HD int exact_floor(const FrameArgs& A, bool round, float y, double cg, double sg, double sv,
                                           double se) {
    const int m = (int)rintf(y);
    // boundary y = m sits at theta = (m - N_b/2 - 1/2) pi / N_b (ROUND) or (m - N_b/2) pi / N_b
    const int h = round ? 2 * m - (NB + 1) : 2 * m - NB;
    return at_or_above<NB>(A, h, cg, sg, sv, se) ? m : max(m - 1, 0);
}

// Direction of a clamped endpoint: the hemisphere edge it was clamped to (side -1 below
// -pi/2, +1 above +pi/2), else the sample's own direction.
SSVB_HD void endpoint_dir(int side, double cg, double sg, double sv, double se, double& dv,
                                             double& de) {
    if (side < 0) {  // theta = -pi/2
        dv = sg;
        de = -cg;
    } else if (side > 0) {  // theta = +pi/2
        dv = -sg;
        de = cg;
    } else {
        dv = sv;
        de = se;
    }
}

// ---------------------------------------------------------------------------------------
// the gather
// ---------------------------------------------------------------------------------------
// MODE_COMPUTE: the pixel's outputs; MODE_PARTIAL: one slice's sums to the partial buffer
// (slice-major order); MODE_LATTICE / MODE_ENDPOINTS: test hooks
enum { MODE_COMPUTE = 0, MODE_LATTICE = 1, MODE_ENDPOINTS = 2, MODE_PARTIAL = 3 };

SSVB_HD void store_background(const FrameArgs& A, int x, int y, int li) {
    if (li != 0) return;
    *(GMEM float*)((GMEM char*)A.ao + (int64_t)y * A.ao_pitch + (int64_t)x * 4) = 1.0f;
    GMEM float* g = (GMEM float*)((GMEM char*)A.gi + (int64_t)y * A.gi_pitch) + 3 * (int64_t)x;
    GMEM float* m = (GMEM float*)((GMEM char*)A.amb + (int64_t)y * A.amb_pitch) + 3 * (int64_t)x;
    g[0] = g[1] = g[2] = 0.0f;
    m[0] = m[1] = m[2] = 0.0f;
    if (A.masks) {
        const int words = A.nd * (A.nb / 32);
        GMEM uint32_t* mk = (GMEM uint32_t*)((GMEM char*)A.masks + (int64_t)y * A.masks_pitch) + (int64_t)x * words;
        for (int i = 0; i < words; ++i) mk[i] = 0u;
    }
}

// One sample of the march: sector range, newly covered sectors, indirect light.
template <int CRIT, bool TINF, int FMT, int NB>
SSVB_HD void march_sample(const FrameArgs& A, const SliceF& S, const ExactLds& L, int t, float zp,
                                             float R, float vx, float vy, float vz, float tp, int s, int o, int X,
                                             int Y, bool ok, float zs, SMask<NB>& B, float& gir, float& gig,
                                             float& gib) {
    constexpr float hi_edge = (float)NB + 0.5f;
    constexpr float guard = kGuard * (NB / 32);
    ok = ok && is_geometry(zs);
    const float of = (float)o;
    const float sk = s > 0 ? (float)NB * kInvPi : -(float)NB * kInvPi;
    // slice-plane coordinates of delta = s_f - p: c along v, h = |delta . e|
    const float c = fmaf(zs, of * (s > 0 ? S.avq : -S.avq), -R * (zs - zp));
    const float h = zs * (of * S.aeq);
    // front and back angles from v (the back sample lies t farther along -v)
    const float af = atan2_pos(h, c);
    const float ab = TINF ? 3.14159265358979324f : atan2_pos(h, c - tp);
    const float yf = fminf(fmaxf(fmaf(af, sk, S.K), 0.5f), hi_edge);
    const float yb = fminf(fmaxf(fmaf(ab, sk, S.K), 0.5f), hi_edge);
    const bool round = CRIT < 0 ? A.criterion == SSVB_HIT_ROUND : CRIT == SSVB_HIT_ROUND;
    int a, b;
    if (round) {
        int kf = (int)floorf(yf), kb = (int)floorf(yb);
        if ((near_integer<NB>(yf) | near_integer<NB>(yb)) && ok) {
            // FP64 decision of the endpoint(s) next to a boundary
            const double zsd = zs, zpd = zp;
            const double lam = (double)(s * o) * 0.0625;
            const double cd = -(zsd - zpd) * L.R[t] + zsd * lam * L.av[t];
            const double he = zsd * lam * L.ae[t];
            const double cg = L.cg[t], sg = L.sg[t];
            if (near_integer<NB>(yf)) kf = exact_floor<NB>(A, round, yf, cg, sg, cd, he);
            if (near_integer<NB>(yb)) {
                if (TINF || isinf(L.tp[t])) kb = exact_floor<NB>(A, round, yb, cg, sg, -1.0, 0.0);
                else kb = exact_floor<NB>(A, round, yb, cg, sg, cd - L.tp[t], he);
            }
        }
        a = min(kf, kb);
        b = max(kf, kb);
    } else {
        // the angular order of the endpoints is fixed by geometry: on the + side the back
        // angle is at or above the front one, on the - side at or below it
        const float lo = s > 0 ? yf : yb, hi = s > 0 ? yb : yf;
        int kf = (int)floorf(yf - 0.5f), kb = (int)floorf(yb - 0.5f);
        const float wf = hi - lo;
        int w = (int)ceilf(fmaxf(wf, 0.0f));
        if ((near_integer<NB>(yf - 0.5f) | near_integer<NB>(yb - 0.5f) | near_integer<NB>(wf)) && ok) {
#pragma clang fp contract(off)
            const double zsd = zs, zpd = zp;
            const double lam = (double)(s * o) * 0.0625;
            const double cd = -(zsd - zpd) * L.R[t] + zsd * lam * L.av[t];
            const double he = zsd * lam * L.ae[t];
            const double cg = L.cg[t], sg = L.sg[t];
            const bool binf = TINF || isinf(L.tp[t]);
            const double bv = binf ? -1.0 : cd - L.tp[t], be = binf ? 0.0 : he;
            if (near_integer<NB>(yf - 0.5f)) kf = exact_floor<NB>(A, round, yf - 0.5f, cg, sg, cd, he);
            if (near_integer<NB>(yb - 0.5f)) kb = exact_floor<NB>(A, round, yb - 0.5f, cg, sg, bv, be);
            if (near_integer<NB>(wf)) {
                // width = ceil of the angle between the two clamped endpoint directions; an
                // endpoint near a hemisphere edge is clamped (or not) exactly
                const float yfr = fmaf(af, sk, S.K), ybr = TINF ? yb : fmaf(ab, sk, S.K);
                int sf = 0, sb = 0;  // +1 above the +pi/2 edge, -1 below the -pi/2 edge
                if (yfr >= hi_edge + guard || (yfr > hi_edge - guard && at_or_above<NB>(A, NB, cg, sg, cd, he))) sf = 1;
                if (yfr <= 0.5f - guard || (yfr < 0.5f + guard && !at_or_above<NB>(A, -NB, cg, sg, cd, he))) sf = -1;
                if (ybr >= hi_edge + guard || (ybr > hi_edge - guard && at_or_above<NB>(A, NB, cg, sg, bv, be))) sb = 1;
                if (ybr <= 0.5f - guard || (ybr < 0.5f + guard && !at_or_above<NB>(A, -NB, cg, sg, bv, be))) sb = -1;
                if (sf != 0 && sf == sb) {
                    w = 0;  // both endpoints on the same edge
                } else {
                    double fv, fe, bv2, be2;
                    endpoint_dir(sf, cg, sg, cd, he, fv, fe);
                    endpoint_dir(sb, cg, sg, bv, be, bv2, be2);
                    const double lv = s > 0 ? fv : bv2, le = s > 0 ? fe : be2;
                    const double hv = s > 0 ? bv2 : fv, hev = s > 0 ? be2 : fe;
                    const int m = max((int)rintf(wf), 0);
                    // rotate the low end by m pi / N_b
                    const GMEM double* hs = (const GMEM double*)A.half_sector + 2 * (2 * m + 2 * NB);
                    const double2 cs = make_double2(hs[0], hs[1]);
                    const double rv = cs.x * lv - cs.y * le, re = cs.y * lv + cs.x * le;
                    w = (rv * hev - re * hv <= 0.0) ? m : m + 1;
                }
            }
        }
        a = min(kf, kb);
        b = min(a + w, NB);
    }
    const SMask<NB> m = ok ? mask_range<NB>(a, b) : mask_none<NB>();
    // newly covered sectors: at 32 sectors m & ~B before B |= m (below); above, cover()
    // updates B and its count at once
    SMask<NB> fresh_m;
    int fresh = 0;
    bool any;
    if constexpr (NB == 32) {
        fresh_m = mask_and_not<NB>(m, B);
        any = mask_any<NB>(fresh_m);
    } else {
        fresh = cover<NB>(B, m);
        any = fresh > 0;
    }
    if (any) {
        // indirect light from the newly covered sectors (Algorithm 1; Section 3.3)
        const float3 nj = load3<FMT < 0 ? -1 : (FMT & 1)>(A.normal, A.normal_pitch, A.normal_ch, A.normal_f16, X, Y);
        const float hs = s > 0 ? h : -h;
        const float ndp = fmaf(S.nv, c, S.ne * hs);
        const float njv = nj.x * vx + nj.y * vy + nj.z * vz;
        const float nje = nj.x * S.ex + nj.y * S.ey + nj.z * S.ez;
        const float ndj = fmaf(njv, c, nje * hs);
        const float w = (float)(NB == 32 ? mask_popc<NB>(fresh_m) : fresh) * (1.0f / (float)NB) *
                        fmaxf(ndp, 0.0f) * fmaxf(-ndj, 0.0f) * rcp_approx(fmaf(c, c, h * h));
        if (w > 0.0f) {
            const float3 cj = load3<FMT < 0 ? -1 : (FMT >> 1)>(A.radiance, A.radiance_pitch, A.radiance_ch,
                                                              A.radiance_f16, X, Y);
            gir = fmaf(w, cj.x, gir);
            gig = fmaf(w, cj.y, gig);
            gib = fmaf(w, cj.z, gib);
        }
    }
    if constexpr (NB == 32) B.w[0] |= m.w[0];
}

// One pixel of the gather.
//  CRIT   hit criterion
//  MODE   compute, or dump the lattice / the FP32 endpoint arguments (test hooks)
//  TINF   thickness is +inf: every back angle is pi, no second atan2
//  FMT    bit 0: normals FP16, bit 1: radiance FP16
// Both sides of a slice advance together, one step per iteration: the + side only
// covers sectors at or above the direction v and the - side only sectors below it, so
// the two never compete for a sector and the interleaving leaves every mask, and every
// newly covered count, as a side-by-side march would produce it.
//  li/lp  this lane's index among the lp lanes that share the pixel (adjacent lanes, lp a
//         power of two); lane li takes slices li, li + lp, ...
//  QUAD   quadratic step distribution
//  FAR    every step is at least one pixel long, so no sample can fall on the centre
//         texel and its test is left out: the offset is then >= 16/16 px along a
//         direction of length >= 4095/4096, while a sample in the centre texel lies
//         within 0.5 px of the centre on both axes, i.e. within 0.71 px
template <int CRIT, int MODE, bool TINF, int FMT, int NB, bool QUAD, bool FAR>
SSVB_HD void gather_pixel_steps(const FrameArgs& A, ExactLds& L, int x, int y, int li, int lp,
                                                   int32_t* dbg_i, float* dbg_f) {
    const int t = thread_index();
    const float zp = depth_load(A, depth_off(A, x, y));
    const bool geom = is_geometry(zp);
    if (MODE == MODE_COMPUTE && !geom) {
        store_background(A, x, y, li);
        return;
    }
    if (MODE == MODE_PARTIAL && !geom) return;  // the reduction writes background pixels
    const float3 n = MODE == MODE_LATTICE ? make_float3(0.0f, 0.0f, 1.0f)
                                          : load3<FMT < 0 ? -1 : (FMT & 1)>(A.normal, A.normal_pitch, A.normal_ch,
                                                                            A.normal_f16, x, y);
    const uint32_t rho = rotation16(A, x, y);

    // step length in 1/16 px: floor(C / z_p) from one IEEE FP32 division, clamped
    float quot = div_rn(A.c_step, geom ? zp : 1.0f);
    quot = fminf(quot, A.q_max_f);
    const int q = max((int)floorf(quot), A.q_min);
    const float tp = fmaf(A.tk, zp, A.t0);

    // view ray of the pixel centre (FP64), its length and the unit vector v to the camera
    const double rpx = ((double)x + 0.5 - (double)A.cx) / (double)A.fx;
    const double rpy = -((double)y + 0.5 - (double)A.cy) / (double)A.fy;
    float R, vx, vy, vz;
    {
        const double Rd = sqrt(rpx * rpx + rpy * rpy + 1.0);
        R = (float)Rd;
        vx = (float)(-rpx / Rd);
        vy = (float)(-rpy / Rd);
        vz = (float)(1.0 / Rd);
        L.R[t] = Rd;
        L.tp[t] = (double)A.t0 + (double)A.tk * (double)zp;
    }

    float ao_acc = 0.0f;
    float gir = 0.0f, gig = 0.0f, gib = 0.0f;
    float amr = 0.0f, amg = 0.0f, amb = 0.0f;
    const int x16 = (x << 16) + 32768, y16 = (y << 16) + 32768;
    const uint32_t own = depth_off(A, x, y);

    for (int i = li; i < A.nd; i += lp) {
        const int k = (int)(((uint32_t)i * 65536u + rho) / (uint32_t)(16 * A.nd));
        const GMEM int* dk = (const GMEM int*)A.lut + 2 * k;
        const int2 D = make_int2(dk[0], dk[1]);
        const int xi8 = (int)jitter8(A, x, y, i);
        const int jit = (q * xi8) >> 8;
        if (MODE == MODE_LATTICE) {
            for (int side = 0; side < 2; ++side) {
                const int s = side ? -1 : 1;
                for (int j = 0; j < A.ns; ++j) {
                    const int o = step_offset<QUAD>(A, q, jit, xi8, j);
                    int32_t* d = dbg_i + ((((int64_t)i * 2 + side) * A.ns + j) * 2);
                    d[0] = lattice_coord(x16, s * o, D.x);
                    d[1] = lattice_coord(y16, s * o, D.y);
                }
            }
            continue;
        }
        const SliceF S = slice_constants<NB>(A, rpx, rpy, D, n, L, t);
        SMask<NB> B = mask_none<NB>();

        // steps are taken kBatch at a time: the depth loads of the whole batch (both
        // sides) are issued first, then the samples are consumed near to far
        for (int j0 = 0; j0 < A.ns; j0 += kBatch) {
            float zs[kBatch][2];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int o = step_offset<QUAD>(A, q, jit, xi8, j0 + u);
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int so = side ? -o : o;
                    const int X = lattice_coord(x16, so, D.x), Y = lattice_coord(y16, so, D.y);
                    const bool ok = j0 + u < A.ns && (unsigned)X < (unsigned)A.W && (unsigned)Y < (unsigned)A.H &&
                                    (FAR || !(X == x && Y == y)) && geom;
                    zs[u][side] = depth_load(A, ok ? depth_off(A, X, Y) : own);
                }
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int j = j0 + u;
                if (j >= A.ns) break;
                const int o = step_offset<QUAD>(A, q, jit, xi8, j);
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int s = side ? -1 : 1;
                    const int so = side ? -o : o;
                    const int X = lattice_coord(x16, so, D.x), Y = lattice_coord(y16, so, D.y);
                    const bool ok = (unsigned)X < (unsigned)A.W && (unsigned)Y < (unsigned)A.H &&
                                    (FAR || !(X == x && Y == y)) && geom;
                    if (MODE == MODE_ENDPOINTS) {
                        const float z = zs[u][side];
                        if (!(ok && is_geometry(z))) continue;
                        const float of = (float)o;
                        const float sk = side ? -(float)NB * kInvPi : (float)NB * kInvPi;
                        const float c = fmaf(z, of * (side ? -S.avq : S.avq), -R * (z - zp));
                        const float h = z * (of * S.aeq);
                        const float af = atan2_pos(h, c);
                        const float ab = atan2_pos(h, c - tp);
                        const float yf = fminf(fmaxf(fmaf(af, sk, S.K), 0.5f), (float)NB + 0.5f);
                        const float yb = fminf(fmaxf(fmaf(ab, sk, S.K), 0.5f), (float)NB + 0.5f);
                        const float lo = fminf(yf, yb), hi = fmaxf(yf, yb);
                        float* d = dbg_f + ((((int64_t)i * 2 + side) * A.ns + j) * 2);
                        const bool round = CRIT < 0 ? A.criterion == SSVB_HIT_ROUND : CRIT == SSVB_HIT_ROUND;
                        d[0] = round ? lo : lo - 0.5f;
                        d[1] = round ? hi : hi - lo;
                    } else {
                        march_sample<CRIT, TINF, FMT, NB>(A, S, L, t, zp, R, vx, vy, vz, tp, s, o, X, Y, ok,
                                                      zs[u][side], B, gir, gig, gib);
                    }
                }
            }
        }
        if (MODE != MODE_COMPUTE && MODE != MODE_PARTIAL) continue;
        ao_acc += 1.0f - (float)(NB == 32 ? mask_popc<NB>(B) : B.n) * (1.0f / (float)NB);
        if (A.masks) {
            GMEM uint32_t* mk = (GMEM uint32_t*)((GMEM char*)A.masks + (int64_t)y * A.masks_pitch) +
                                (int64_t)x * A.nd * SMask<NB>::W;
#pragma unroll
            for (int k = 0; k < SMask<NB>::W; ++k) mk[i * SMask<NB>::W + k] = B.w[k];
        }
        // directionally occluded ambient (Section 3.2)
        const int per = NB / A.na;
        for (int kk = 0; kk < A.na; ++kk) {
            const SMask<NB> open = mask_and_not<NB>(mask_range<NB>(kk * per, (kk + 1) * per), B);
            if (!mask_any<NB>(open)) continue;
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
            const float fr = (float)mask_popc<NB>(open) * (1.0f / (float)NB);
            amr = fmaf(fr, Lr, amr);
            amg = fmaf(fr, Lg, amg);
            amb = fmaf(fr, Lb, amb);
        }
    }
    if (MODE == MODE_PARTIAL) {
        // slice li's sums (the caller runs one slice per thread, lp = N_d; dbg_f is the
        // partial buffer)
        GMEM PartialQuad* pr = (GMEM PartialQuad*)((GMEM float*)dbg_f + partial_off(A, x, y, li));
        pr[0] = PartialQuad{ao_acc, gir, gig, gib};
        pr[1] = PartialQuad{amr, amg, amb, 0.0f};
        return;
    }
    if (MODE != MODE_COMPUTE) return;
    // sum the lanes of the pixel (butterfly: every lane ends with the same value)
    for (int off = 1; off < lp; off <<= 1) {
        ao_acc += lane_xor(ao_acc, off);
        gir += lane_xor(gir, off);
        gig += lane_xor(gig, off);
        gib += lane_xor(gib, off);
        amr += lane_xor(amr, off);
        amg += lane_xor(amg, off);
        amb += lane_xor(amb, off);
    }
    if (li != 0) return;
    const float inv_nd = 1.0f / (float)A.nd;
    *(GMEM float*)((GMEM char*)A.ao + (int64_t)y * A.ao_pitch + (int64_t)x * 4) = ao_acc * inv_nd;
    GMEM float* g = (GMEM float*)((GMEM char*)A.gi + (int64_t)y * A.gi_pitch) + 3 * (int64_t)x;
    g[0] = gir * inv_nd;
    g[1] = gig * inv_nd;
    g[2] = gib * inv_nd;
    GMEM float* m = (GMEM float*)((GMEM char*)A.amb + (int64_t)y * A.amb_pitch) + 3 * (int64_t)x;
    m[0] = amr * inv_nd;
    m[1] = amg * inv_nd;
    m[2] = amb * inv_nd;
}

// The step distribution is uniform per frame: decide it once per pixel, outside the
// step loops (inside them the compiler would evaluate both placements and select).
template <int CRIT, int MODE, bool TINF, int FMT, int NB = 32>
SSVB_HD void gather_pixel(const FrameArgs& A, ExactLds& L, int x, int y, int li, int lp,
                                             int32_t* dbg_i, float* dbg_f) {
    // uniform steps are q (j + 1) + jitter >= q >= q_min 1/16 px long
    if (A.step_dist == SSVB_STEPS_QUADRATIC)
        gather_pixel_steps<CRIT, MODE, TINF, FMT, NB, true, false>(A, L, x, y, li, lp, dbg_i, dbg_f);
    else if (A.q_min >= 16)
        gather_pixel_steps<CRIT, MODE, TINF, FMT, NB, false, true>(A, L, x, y, li, lp, dbg_i, dbg_f);
    else
        gather_pixel_steps<CRIT, MODE, TINF, FMT, NB, false, false>(A, L, x, y, li, lp, dbg_i, dbg_f);
}

// Second pass of the slice-major order: the computed pixel (x, y)'s outputs from its slices'
// sums, added in slice order (the AO sums are those of the one-pass kernel, bit for bit);
// a background pixel gets AO 1, GI 0, ambient 0 and empty masks.
SSVB_HD void reduce_pixel(const FrameArgs& A, const float* partial, int x, int y) {
    if (!is_geometry(depth_load(A, depth_off(A, x, y)))) {
        store_background(A, x, y, 0);
        return;
    }
    float ao_acc = 0.0f, gir = 0.0f, gig = 0.0f, gib = 0.0f, amr = 0.0f, amg = 0.0f, amb = 0.0f;
    for (int i = 0; i < A.nd; ++i) {
        const GMEM PartialQuad* p = (const GMEM PartialQuad*)((const GMEM float*)partial + partial_off(A, x, y, i));
        const PartialQuad a = p[0], b = p[1];
        ao_acc += a.x;
        gir += a.y, gig += a.z, gib += a.w;
        amr += b.x, amg += b.y, amb += b.z;
    }
    const float inv_nd = 1.0f / (float)A.nd;
    *(GMEM float*)((GMEM char*)A.ao + (int64_t)y * A.ao_pitch + (int64_t)x * 4) = ao_acc * inv_nd;
    GMEM float* g = (GMEM float*)((GMEM char*)A.gi + (int64_t)y * A.gi_pitch) + 3 * (int64_t)x;
    g[0] = gir * inv_nd;
    g[1] = gig * inv_nd;
    g[2] = gib * inv_nd;
    GMEM float* m = (GMEM float*)((GMEM char*)A.amb + (int64_t)y * A.amb_pitch) + 3 * (int64_t)x;
    m[0] = amr * inv_nd;
    m[1] = amg * inv_nd;
    m[2] = amb * inv_nd;
}

// Half resolution: every pixel with an odd coordinate takes the average of its 1, 2 or
// 4 nearest computed (even, even) pixels, weighted bilinear x (1e-3 + exp(-(dz /
// (0.05 z))^2)); background neighbours are left out; a background pixel, or one with no
// computed foreground neighbour, gets AO = 1, GI = 0, ambient = 0.  Reads only computed
// pixels and writes only the others, so it works in place on the outputs.
SSVB_HD void upsample_pixel(const FrameArgs& A, int x, int y) {
    if (x >= A.W || y >= A.H || ((x | y) & 1) == 0) return;
    const float z = depth_load(A, depth_off(A, x, y));
    float sw = 0.0f, sa = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, m0 = 0.0f, m1 = 0.0f, m2 = 0.0f;
    if (is_geometry(z)) {
        const int x0 = x & ~1, y0 = y & ~1;
        const int nx = (x & 1) && x + 1 < A.W ? 2 : 1, ny = (y & 1) && y + 1 < A.H ? 2 : 1;
        const float bx = nx == 2 ? 0.5f : 1.0f, by = ny == 2 ? 0.5f : 1.0f;
        const float inv = 1.0f / (0.05f * z);
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                const int xn = x0 + 2 * i, yn = y0 + 2 * j;
                const float zn = depth_load(A, depth_off(A, xn, yn));
                if (!is_geometry(zn)) continue;
                const float d = (z - zn) * inv;
                const float w = bx * by * (1e-3f + expf(-d * d));
                const GMEM float* g = (const GMEM float*)((const GMEM char*)A.gi + (int64_t)yn * A.gi_pitch) + 3 * xn;
                const GMEM float* m = (const GMEM float*)((const GMEM char*)A.amb + (int64_t)yn * A.amb_pitch) + 3 * xn;
                sw += w;
                sa = fmaf(w, *(const GMEM float*)((const GMEM char*)A.ao + (int64_t)yn * A.ao_pitch + 4 * xn), sa);
                s0 = fmaf(w, g[0], s0);
                s1 = fmaf(w, g[1], s1);
                s2 = fmaf(w, g[2], s2);
                m0 = fmaf(w, m[0], m0);
                m1 = fmaf(w, m[1], m1);
                m2 = fmaf(w, m[2], m2);
            }
        }
    }
    float ao = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    if (sw > 0.0f) {
        const float r = 1.0f / sw;
        ao = sa * r;
        g0 = s0 * r, g1 = s1 * r, g2 = s2 * r;
        a0 = m0 * r, a1 = m1 * r, a2 = m2 * r;
    }
    *(GMEM float*)((GMEM char*)A.ao + (int64_t)y * A.ao_pitch + 4 * (int64_t)x) = ao;
    GMEM float* g = (GMEM float*)((GMEM char*)A.gi + (int64_t)y * A.gi_pitch) + 3 * (int64_t)x;
    g[0] = g0, g[1] = g1, g[2] = g2;
    GMEM float* m = (GMEM float*)((GMEM char*)A.amb + (int64_t)y * A.amb_pitch) + 3 * (int64_t)x;
    m[0] = a0, m[1] = a1, m[2] = a2;
}

}  // namespace ssvb
