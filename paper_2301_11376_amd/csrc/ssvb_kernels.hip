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

#include "ssvb_internal.h"

namespace ssvb {

constexpr float kInvPi32 = 10.185916357881302f;  // 32 / pi
constexpr double kInvPi32d = 10.185916357881301489;
constexpr double kPi = 3.141592653589793238;
constexpr float kGuard = 1.0f / 32768.0f;       // sectors; ~3e-6 rad

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

__device__ __forceinline__ float3 load3(const char* base, int64_t pitch, int ch, int f16, int x, int y) {
    const char* row = base + (int64_t)y * pitch;
    if (f16) {
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

// ---------------------------------------------------------------------------------------
// the gather
// ---------------------------------------------------------------------------------------
enum { MODE_COMPUTE = 0, MODE_LATTICE = 1, MODE_ENDPOINTS = 2 };

template <int CRIT, int MODE>
__device__ __forceinline__ void gather_pixel(const FrameArgs& A, int x, int y, int32_t* dbg_i, float* dbg_f) {
    const float zp = depth_at(A, x, y);
    const bool geom = is_geometry(zp);
    if (MODE == MODE_COMPUTE && !geom) {
        *(float*)((char*)A.ao + (int64_t)y * A.ao_pitch + (int64_t)x * 4) = 1.0f;
        float* g = (float*)((char*)A.gi + (int64_t)y * A.gi_pitch) + 3 * (int64_t)x;
        float* m = (float*)((char*)A.amb + (int64_t)y * A.amb_pitch) + 3 * (int64_t)x;
        g[0] = g[1] = g[2] = 0.0f;
        m[0] = m[1] = m[2] = 0.0f;
        if (A.masks) {
            uint32_t* mk = (uint32_t*)((char*)A.masks + (int64_t)y * A.masks_pitch) + (int64_t)x * A.nd;
            for (int i = 0; i < A.nd; ++i) mk[i] = 0u;
        }
        return;
    }
    const float3 n = load3(A.normal, A.normal_pitch, A.normal_ch, A.normal_f16, x, y);
    const uint32_t rho = rotation16(A, x, y);

    // step length in 1/16 px: floor(C / z_p) from one IEEE FP32 division, clamped
    float quot = __fdiv_rn(A.c_step, geom ? zp : 1.0f);
    quot = fminf(quot, A.q_max_f);
    const int q = max((int)floorf(quot), A.q_min);
    const float tp = fmaf(A.tk, zp, A.t0);

    Frame64 F;
    pixel_ray64(A, x, y, F);
    const float R = (float)F.R;
    const float vx = (float)F.vx, vy = (float)F.vy, vz = (float)F.vz;

    float ao_acc = 0.0f;
    float gir = 0.0f, gig = 0.0f, gib = 0.0f;
    float amr = 0.0f, amg = 0.0f, amb = 0.0f;
    const int x16 = (x << 16) + 32768, y16 = (y << 16) + 32768;

    for (int i = 0; i < A.nd; ++i) {
        const int k = (int)(((uint32_t)i * 65536u + rho) / (uint32_t)(16 * A.nd));
        const int2 D = A.lut[k];
        slice_frame64(A, D.x, D.y, n, F);
        const float ex = (float)F.ex, ey = (float)F.ey, ez = (float)F.ez;
        const float nv = (float)F.nv, ne = (float)F.ne;
        const float K = (float)(16.5 - F.gamma * kInvPi32d);
        const float avq = (float)(F.av / 16.0), aeq = (float)(F.ae / 16.0);
        const int jit = (q * (int)jitter8(A, x, y, i)) >> 8;
        uint32_t B = 0u;

        for (int side = 0; side < 2; ++side) {
            const int s = side ? -1 : 1;
            const int sDx = s * D.x, sDy = s * D.y;
            const float sk = s * kInvPi32;
            const float savq = s * avq;
            for (int j = 0; j < A.ns; ++j) {
                const int o = q * (j + 1) + jit;
                const int X = (x16 + o * sDx) >> 16;
                const int Y = (y16 + o * sDy) >> 16;
                if (MODE == MODE_LATTICE) {
                    int32_t* d = dbg_i + ((((int64_t)i * 2 + side) * A.ns + j) * 2);
                    d[0] = X;
                    d[1] = Y;
                    continue;
                }
                if ((unsigned)X >= (unsigned)A.W || (unsigned)Y >= (unsigned)A.H || (X == x && Y == y) || !geom)
                    continue;
                const float zs = depth_at(A, X, Y);
                if (!is_geometry(zs)) continue;
                const float of = (float)o;
                // slice-plane coordinates of delta = s_f - p: c along v, h along e (|h|)
                const float c = fmaf(zs, of * savq, -R * (zs - zp));
                const float h = zs * (of * aeq);
                // front and back angles from v (back sample t farther along -v)
                const float af = atan2f(h, c);
                const float ab = atan2f(h, c - tp);
                float yf = fminf(fmaxf(fmaf(af, sk, K), 0.5f), 32.5f);
                float yb = fminf(fmaxf(fmaf(ab, sk, K), 0.5f), 32.5f);
                const float lo = fminf(yf, yb), hi = fmaxf(yf, yb);
                if (MODE == MODE_ENDPOINTS) {
                    float* d = dbg_f + ((((int64_t)i * 2 + side) * A.ns + j) * 2);
                    if (CRIT == SSVB_HIT_ROUND) {
                        d[0] = lo;
                        d[1] = hi;
                    } else {
                        d[0] = lo - 0.5f;
                        d[1] = hi - lo;
                    }
                    continue;
                }
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
                if (near) {
                    const int2 ab64 = decide64<CRIT>(A, x, y, zp, zs, s * o, D.x, D.y, n);
                    a = ab64.x;
                    b = ab64.y;
                }
                const uint32_t m = range_bits(a, b);
                const uint32_t fresh = m & ~B;
                if (fresh) {
                    // indirect light from the newly covered sectors (Algorithm 1; Section 3.3)
                    const float3 nj = load3(A.normal, A.normal_pitch, A.normal_ch, A.normal_f16, X, Y);
                    const float3 cj = load3(A.radiance, A.radiance_pitch, A.radiance_ch, A.radiance_f16, X, Y);
                    const float hs = s * h;
                    const float ndp = fmaf(nv, c, ne * hs);
                    const float njv = nj.x * vx + nj.y * vy + nj.z * vz;
                    const float nje = nj.x * ex + nj.y * ey + nj.z * ez;
                    const float ndj = fmaf(njv, c, nje * hs);
                    const float w = (float)__popc(fresh) * (1.0f / 32.0f) * fmaxf(ndp, 0.0f) * fmaxf(-ndj, 0.0f) /
                                    fmaf(c, c, h * h);
                    gir = fmaf(w, cj.x, gir);
                    gig = fmaf(w, cj.y, gig);
                    gib = fmaf(w, cj.z, gib);
                }
                B |= m;
            }
        }
        if (MODE != MODE_COMPUTE) continue;
        ao_acc += 1.0f - (float)__popc(B) * (1.0f / 32.0f);
        if (A.masks) {
            uint32_t* mk = (uint32_t*)((char*)A.masks + (int64_t)y * A.masks_pitch) + (int64_t)x * A.nd;
            mk[i] = B;
        }
        // directionally occluded ambient (Section 3.2)
        float cg = 1.0f, sg = 0.0f;
        {
            const double g2 = F.nv * F.nv + F.ne * F.ne;
            if (g2 >= 1e-12) {
                const double ig = 1.0 / sqrt(g2);
                cg = (float)(F.nv * ig);
                sg = (float)(F.ne * ig);
            }
        }
        const int per = 32 / A.na;
        for (int kk = 0; kk < A.na; ++kk) {
            const uint32_t open = ~B & range_bits(kk * per, (kk + 1) * per);
            if (!open) continue;
            const float cps = cg * A.amb_cb[kk] - sg * A.amb_sb[kk];
            const float sps = sg * A.amb_cb[kk] + cg * A.amb_sb[kk];
            const float dvx = cps * vx + sps * ex, dvy = cps * vy + sps * ey, dvz = cps * vz + sps * ez;
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
            const float* S = A.sh;
            const float Lr = b0 * S[0] + b1 * S[3] + b2 * S[6] + b3 * S[9] + b4 * S[12] + b5 * S[15] + b6 * S[18] +
                             b7 * S[21] + b8 * S[24];
            const float Lg = b0 * S[1] + b1 * S[4] + b2 * S[7] + b3 * S[10] + b4 * S[13] + b5 * S[16] +
                             b6 * S[19] + b7 * S[22] + b8 * S[25];
            const float Lb = b0 * S[2] + b1 * S[5] + b2 * S[8] + b3 * S[11] + b4 * S[14] + b5 * S[17] +
                             b6 * S[20] + b7 * S[23] + b8 * S[26];
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
}

template <int CRIT>
__global__ __launch_bounds__(256) void gather_plain(FrameArgs A) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= A.W || y >= A.H) return;
    gather_pixel<CRIT, MODE_COMPUTE>(A, x, y, nullptr, nullptr);
}

__global__ __launch_bounds__(256) void debug_lattice(FrameArgs A, int32_t* out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= A.W || y >= A.H) return;
    int32_t* d = out + ((int64_t)y * A.W + x) * (int64_t)A.nd * 2 * A.ns * 2;
    gather_pixel<SSVB_HIT_ROUND, MODE_LATTICE>(A, x, y, d, nullptr);
}

template <int CRIT>
__global__ __launch_bounds__(256) void debug_endpoints(FrameArgs A, float* out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= A.W || y >= A.H) return;
    float* d = out + ((int64_t)y * A.W + x) * (int64_t)A.nd * 2 * A.ns * 2;
    gather_pixel<CRIT, MODE_ENDPOINTS>(A, x, y, nullptr, d);
}

// ---------------------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------------------
static dim3 plain_grid(const FrameArgs& A, dim3 block) {
    return dim3((A.W + block.x - 1) / block.x, (A.H + block.y - 1) / block.y);
}

hipError_t launch_plain(const FrameArgs& A, hipStream_t stream) {
    const dim3 block(16, 16);
    const dim3 grid = plain_grid(A, block);
    if (A.criterion == SSVB_HIT_ROUND)
        hipLaunchKernelGGL(gather_plain<SSVB_HIT_ROUND>, grid, block, 0, stream, A);
    else
        hipLaunchKernelGGL(gather_plain<SSVB_HIT_PSEUDOCODE>, grid, block, 0, stream, A);
    return hipGetLastError();
}

hipError_t launch_debug_lattice(const FrameArgs& A, int32_t* out, hipStream_t stream) {
    const dim3 block(16, 16);
    hipLaunchKernelGGL(debug_lattice, plain_grid(A, block), block, 0, stream, A, out);
    return hipGetLastError();
}

hipError_t launch_debug_endpoints(const FrameArgs& A, float* out, hipStream_t stream) {
    const dim3 block(16, 16);
    if (A.criterion == SSVB_HIT_ROUND)
        hipLaunchKernelGGL(debug_endpoints<SSVB_HIT_ROUND>, plain_grid(A, block), block, 0, stream, A, out);
    else
        hipLaunchKernelGGL(debug_endpoints<SSVB_HIT_PSEUDOCODE>, plain_grid(A, block), block, 0, stream, A, out);
    return hipGetLastError();
}

}  // namespace ssvb
