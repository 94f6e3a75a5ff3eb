// gfx950 kernels of the visibility-bitmask gather: the persistent single-frame and batch
// kernels (per-XCD tile queues with stealing), the half-resolution upsampling, the
// multi-bounce injection, the test hooks and their host-side launchers.  The per-pixel
// code they run (Algorithm 1 with the ambient split of Section 3.2) is in ssvb_pixel.h.
#include <math.h>

#include <algorithm>

#include "ssvb_pixel.h"

namespace ssvb {

// The XCD this wave runs on (hardware register XCC_ID; the die's own L2 serves it).
__device__ __forceinline__ int hw_xcd() {
    unsigned id;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(id));
    return (int)(id & (kXcds - 1));
}

// Next item of queue `q` for the whole workgroup (uniform).
__device__ __forceinline__ uint32_t grab(uint32_t* q, uint32_t* s_item) {
    if (threadIdx.x == 0) *s_item = atomicAdd(q, 1u);
    __syncthreads();
    const uint32_t item = __builtin_amdgcn_readfirstlane(*s_item);
    __syncthreads();
    return item;
}

// One frame, persistent workgroups.  The frame's tile walk is cut into 8 equal runs,
// run k queued for XCD k (its tiles stay in that die's L2); a workgroup drains the queue
// of its own XCD first and then takes what is left in the others, so dies that finish
// early help the slow ones.  q[0..7] are the queue heads, q[8] counts finished
// workgroups: the last one to finish sets all nine back to zero for the next launch.
template <int CRIT, bool TINF, int FMT, int NB = 32>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void gather_frame(
    FrameArgs A, uint32_t* __restrict__ q) {
    __shared__ ExactLds L;
    __shared__ uint32_t s_item;
    // the frame constants are read from the kernel-argument segment on every tile: an
    // opaque pointer keeps the compiler from holding tile-invariant values in registers
    // across the tile loop (which would cost occupancy)
    typedef const __attribute__((address_space(4))) FrameArgs* ConstArgs;  // scalar-loadable
    const ConstArgs args = (ConstArgs)__builtin_amdgcn_kernarg_segment_ptr();
    const uint32_t nt = (uint32_t)A.tiles_x * (uint32_t)A.tiles_y;
    const int home = hw_xcd();
    for (int qi = 0; qi < kXcds; ++qi) {
        const int k = (home + qi) & (kXcds - 1);
        uint32_t first, count;
        xcd_run(nt, k, first, count);
        for (;;) {
            const uint32_t item = grab(&q[k], &s_item);
            if (item >= count) break;
            ConstArgs ap = args;
            asm volatile("" : "+s"(ap));
            const FrameArgs& F = *(const FrameArgs*)ap;
            int tx, ty, x, y, li;
            walk_tile(F, first + item, tx, ty);
            tile_pixel(F, tx, ty, (int)threadIdx.x, x, y, li);
            if ((unsigned)x < (unsigned)F.W && (unsigned)y < (unsigned)F.H) gather_pixel<CRIT, MODE_COMPUTE, TINF, FMT, NB>(F, L, x, y, li, F.lp, nullptr, nullptr);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&q[kXcds], 1u) == gridDim.x - 1) {
            for (int k = 0; k <= kXcds; ++k) atomicExch(&q[k], 0u);
        }
    }
}

// One frame in slice-major order (A.lp = 1): the work items of XCD k's run of tiles are
// (tile, slice) pairs, slice by slice over chunks of `chunk` tiles, queued for XCD k with
// the same stealing as gather_frame; each item runs one slice of its tile's pixels and
// writes that slice's sums to `partial` (reduce_slices then adds them).  Criterion and
// element types are taken at run time (the batch kernel's instance).
template <int NB>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void gather_slices(
    FrameArgs A, uint32_t* __restrict__ q, float* __restrict__ partial, uint32_t chunk) {
    __shared__ ExactLds L;
    __shared__ uint32_t s_item;
    typedef const __attribute__((address_space(4))) FrameArgs* ConstArgs;
    const ConstArgs args = (ConstArgs)__builtin_amdgcn_kernarg_segment_ptr();
    const uint32_t nt = (uint32_t)A.tiles_x * (uint32_t)A.tiles_y;
    const int home = hw_xcd();
    for (int qi = 0; qi < kXcds; ++qi) {
        const int k = (home + qi) & (kXcds - 1);
        uint32_t first, count;
        xcd_run(nt, k, first, count);
        for (;;) {
            const uint32_t item = grab(&q[k], &s_item);
            if (item >= count * (uint32_t)A.nd) break;
            ConstArgs ap = args;
            asm volatile("" : "+s"(ap));
            const FrameArgs& F = *(const FrameArgs*)ap;
            uint32_t tile;
            int slice, tx, ty, x, y, li;
            slice_item(chunk, F.nd, count, item, tile, slice);
            walk_tile(F, first + tile, tx, ty);
            tile_pixel(F, tx, ty, (int)threadIdx.x, x, y, li);
            if ((unsigned)x < (unsigned)F.W && (unsigned)y < (unsigned)F.H)
                gather_pixel<-1, MODE_PARTIAL, false, -1, NB>(F, L, x, y, slice, F.nd, nullptr, partial);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&q[kXcds], 1u) == gridDim.x - 1) {
            for (int k = 0; k <= kXcds; ++k) atomicExch(&q[k], 0u);
        }
    }
}

// Second pass of the slice-major order: one thread per computed pixel (16 x 16 blocks of
// the computed grid).
__global__ __launch_bounds__(kBlock) void reduce_slices(FrameArgs A, const float* __restrict__ partial) {
    const int u = (int)(blockIdx.x * 16 + threadIdx.x % 16), v = (int)(blockIdx.y * 16 + threadIdx.x / 16);
    const int gw = (A.W + A.sub - 1) / A.sub, gh = (A.H + A.sub - 1) / A.sub;
    if (u < gw && v < gh) reduce_pixel(A, partial, u * A.sub, v * A.sub);
}

__global__ __launch_bounds__(kBlock) void debug_lattice(FrameArgs A, int32_t* out) {
    __shared__ ExactLds L;
    const int x = blockIdx.x * 16 + (int)(threadIdx.x % 16u);
    const int y = blockIdx.y * 16 + (int)(threadIdx.x / 16u);
    if (x >= A.W || y >= A.H) return;
    int32_t* d = out + ((int64_t)y * A.W + x) * (int64_t)A.nd * 2 * A.ns * 2;
    gather_pixel<SSVB_HIT_ROUND, MODE_LATTICE, false, 0>(A, L, x, y, 0, 1, d, nullptr);
}

template <int CRIT, int FMT>
__global__ __launch_bounds__(kBlock) void debug_endpoints(FrameArgs A, float* out) {
    __shared__ ExactLds L;
    const int x = blockIdx.x * 16 + (int)(threadIdx.x % 16u);
    const int y = blockIdx.y * 16 + (int)(threadIdx.x / 16u);
    if (x >= A.W || y >= A.H) return;
    float* d = out + ((int64_t)y * A.W + x) * (int64_t)A.nd * 2 * A.ns * 2;
    gather_pixel<CRIT, MODE_ENDPOINTS, false, FMT>(A, L, x, y, 0, 1, nullptr, d);
}

// Persistent kernel over a batch of frames; workgroup b runs on XCD b mod 8.  Criterion,
// element types and thickness are taken per frame at run time.  One instance per mask
// width: an instance skips the frames of the other width, so the 32-sector instance keeps
// its register budget.  The frames' tile walks form one list cut into 8 runs of equal
// sample cost, one per XCD; a workgroup drains its own run, then steals from the others.
// Every claim returns a tile until the list is exhausted, so frames of a few hundred tiles
// cost no more than their work (with queues per frame every workgroup would pass over
// every queue of every frame).
template <int NB>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void gather_batch(
    const BatchDesc* __restrict__ D, uint32_t* __restrict__ queues) {
    __shared__ ExactLds L;
    __shared__ uint32_t s_item;
    const int home = hw_xcd();
    const int w = NB == 128 ? 1 : 0;
    if (D->pn[w] == 0) return;
    int j = 0;  // frame of the last tile taken: runs are walked in increasing order
    for (int qi = 0; qi < kXcds; ++qi) {
        const int k = (home + qi) & (kXcds - 1);
        const uint32_t first = D->split[w][k];
        const uint32_t count = D->split[w][k + 1] - first;
        for (;;) {
            const uint32_t item = grab(&queues[w * kXcds + k], &s_item);
            if (item >= count) break;
            const uint32_t g = first + item;
            j = batch_frame(*D, w, g, j);
            const FrameArgs& A = D->frames[D->plist[w][j]];
            int tx, ty, x, y, li;
            walk_tile(A, g - D->prefix[w][j], tx, ty);
            tile_pixel(A, tx, ty, (int)threadIdx.x, x, y, li);
            if ((unsigned)x < (unsigned)A.W && (unsigned)y < (unsigned)A.H) gather_pixel<-1, MODE_COMPUTE, false, -1, NB>(A, L, x, y, li, A.lp, nullptr, nullptr);
        }
    }
}

__global__ __launch_bounds__(kBlock) void upsample_half(FrameArgs A) {
    upsample_pixel(A, (int)(blockIdx.x * 16 + threadIdx.x % 16), (int)(blockIdx.y * 16 + threadIdx.x / 16));
}

// The same pass over every half-resolution frame of a batch: a fixed grid whose blocks
// stride over each frame's 16 x 16 pixel blocks.
__global__ __launch_bounds__(kBlock) void upsample_batch(const BatchDesc* __restrict__ D) {
    const int n = D->n_frames;
    for (int f = 0; f < n; ++f) {
        const FrameArgs& A = D->frames[f];
        if (A.sub != 2) continue;
        const int bx = (A.W + 15) / 16, nblk = bx * ((A.H + 15) / 16);
        for (int b = (int)blockIdx.x; b < nblk; b += (int)gridDim.x)
            upsample_pixel(A, (b % bx) * 16 + (int)(threadIdx.x % 16), (b / bx) * 16 + (int)(threadIdx.x / 16));
    }
}

// Multi-bounce: next = direct + gain * albedo * gi per pixel and RGB channel (FP32
// arithmetic); one thread per pixel, each element read before it is written, so `next`
// may be `direct`.
struct BounceArgs {
    const char* direct;
    const char* albedo;
    const float* gi;
    char* next;
    int64_t direct_pitch, albedo_pitch, gi_pitch, next_pitch;
    int32_t W, H, direct_ch, albedo_ch, next_ch;
    int32_t direct_f16, albedo_f16, next_f16;
    float gain;
};

__global__ __launch_bounds__(kBlock) void inject_bounce(BounceArgs B) {
    const int x = (int)(blockIdx.x * 64 + threadIdx.x % 64), y = (int)(blockIdx.y * 4 + threadIdx.x / 64);
    if (x >= B.W || y >= B.H) return;
    const float3 d = load3<-1>(B.direct, B.direct_pitch, B.direct_ch, B.direct_f16, x, y);
    const float3 a = load3<-1>(B.albedo, B.albedo_pitch, B.albedo_ch, B.albedo_f16, x, y);
    const GMEM float* g = (const GMEM float*)((const GMEM char*)B.gi + (int64_t)y * B.gi_pitch) + 3 * (int64_t)x;
    const float r0 = fmaf(B.gain * a.x, g[0], d.x), r1 = fmaf(B.gain * a.y, g[1], d.y),
                r2 = fmaf(B.gain * a.z, g[2], d.z);
    GMEM char* row = (GMEM char*)B.next + (int64_t)y * B.next_pitch;
    if (B.next_f16) {
        GMEM _Float16* o = (GMEM _Float16*)row + (int64_t)x * B.next_ch;
        if (B.next_ch == 4) {
            const GMEM _Float16* ds = (const GMEM _Float16*)((const GMEM char*)B.direct + (int64_t)y * B.direct_pitch);
            const GMEM float* df = (const GMEM float*)((const GMEM char*)B.direct + (int64_t)y * B.direct_pitch);
            o[3] = B.direct_f16 ? ds[4 * x + 3] : (_Float16)df[4 * x + 3];
        }
        o[0] = (_Float16)r0, o[1] = (_Float16)r1, o[2] = (_Float16)r2;
    } else {
        GMEM float* o = (GMEM float*)row + (int64_t)x * B.next_ch;
        if (B.next_ch == 4) {
            const GMEM _Float16* ds = (const GMEM _Float16*)((const GMEM char*)B.direct + (int64_t)y * B.direct_pitch);
            const GMEM float* df = (const GMEM float*)((const GMEM char*)B.direct + (int64_t)y * B.direct_pitch);
            o[3] = B.direct_f16 ? (float)ds[4 * x + 3] : df[4 * x + 3];
        }
        o[0] = r0, o[1] = r1, o[2] = r2;
    }
}

__global__ void reset_queues(uint32_t* q) {
    for (int i = (int)threadIdx.x; i < kBatchQueues; i += (int)blockDim.x) q[i] = 0u;
}

// ---------------------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------------------
hipError_t enqueue_batch(const BatchDesc* d_desc, const BatchDesc* h_desc, uint32_t* d_queues, const int grid[2],
                         int kinds, hipStream_t s) {
    hipError_t e = hipMemcpyAsync((void*)d_desc, h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_queues, dim3(1), dim3(256), 0, s, d_queues);
    if (kinds & kBatch32) hipLaunchKernelGGL(gather_batch<32>, dim3(grid[0]), dim3(kBlock), 0, s, d_desc, d_queues);
    if (kinds & kBatch128) hipLaunchKernelGGL(gather_batch<128>, dim3(grid[1]), dim3(kBlock), 0, s, d_desc, d_queues);
    if (kinds & kBatchHalf) hipLaunchKernelGGL(upsample_batch, dim3(grid[0]), dim3(kBlock), 0, s, d_desc);
    return hipGetLastError();
}

int batch_blocks_per_cu(int nb) {
    int n = 0;
    const hipError_t e = nb == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gather_batch<128>, kBlock, 0)
                                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gather_batch<32>, kBlock, 0);
    return e == hipSuccess && n >= 1 ? n : 2;
}
static dim3 grid16(const FrameArgs& A) { return dim3((A.W + 15) / 16, (A.H + 15) / 16); }

template <int CRIT, bool TINF, int FMT, int NB = 32>
static void launch_main(const FrameArgs& A, uint32_t* q, int grid, hipStream_t stream) {
    // no more workgroups than the frame has tiles (rounded to whole XCD rounds)
    const uint32_t nt = (uint32_t)A.tiles_x * A.tiles_y;
    const uint32_t need = kXcds * ((nt + kXcds - 1) / kXcds);
    const uint32_t nwg = need < (uint32_t)grid ? need : (uint32_t)grid;
    hipLaunchKernelGGL((gather_frame<CRIT, TINF, FMT, NB>), dim3(nwg), dim3(kBlock), 0, stream, A, q);
}

template <int CRIT, bool TINF>
static void launch_fmt(const FrameArgs& A, uint32_t* q, int grid, hipStream_t stream) {
    switch (A.normal_f16 | (A.radiance_f16 << 1)) {
        case 0: launch_main<CRIT, TINF, 0>(A, q, grid, stream); break;
        case 1: launch_main<CRIT, TINF, 1>(A, q, grid, stream); break;
        case 2: launch_main<CRIT, TINF, 2>(A, q, grid, stream); break;
        default: launch_main<CRIT, TINF, 3>(A, q, grid, stream); break;
    }
}

hipError_t launch_plain(const FrameArgs& A, uint32_t* queues, int grid, hipStream_t stream) {
    const bool tinf = isinf(A.t0);
    if (A.nb == 128) {
        // 128 sectors: one kernel for the common case (ROUND, finite thickness, FP32), one
        // that decides criterion and element types at run time
        if (A.criterion == SSVB_HIT_ROUND && !tinf && !A.normal_f16 && !A.radiance_f16)
            launch_main<SSVB_HIT_ROUND, false, 0, 128>(A, queues, grid, stream);
        else
            launch_main<-1, false, -1, 128>(A, queues, grid, stream);
        return hipGetLastError();
    }
    if (A.criterion == SSVB_HIT_ROUND) {
        if (tinf) launch_fmt<SSVB_HIT_ROUND, true>(A, queues, grid, stream);
        else launch_fmt<SSVB_HIT_ROUND, false>(A, queues, grid, stream);
    } else {
        if (tinf) launch_fmt<SSVB_HIT_PSEUDOCODE, true>(A, queues, grid, stream);
        else launch_fmt<SSVB_HIT_PSEUDOCODE, false>(A, queues, grid, stream);
    }
    return hipGetLastError();
}

hipError_t launch_slices(const FrameArgs& A, uint32_t* queues, int grid, float* partial, uint32_t chunk,
                         hipStream_t stream) {
    // no more workgroups than the frame has items (rounded to whole XCD rounds)
    const uint64_t items = (uint64_t)A.tiles_x * A.tiles_y * (uint64_t)A.nd;
    const uint64_t need = kXcds * ((items + kXcds - 1) / kXcds);
    const uint32_t nwg = need < (uint64_t)grid ? (uint32_t)need : (uint32_t)grid;
    if (A.nb == 128)
        hipLaunchKernelGGL(gather_slices<128>, dim3(nwg), dim3(kBlock), 0, stream, A, queues, partial, chunk);
    else
        hipLaunchKernelGGL(gather_slices<32>, dim3(nwg), dim3(kBlock), 0, stream, A, queues, partial, chunk);
    const int gw = (A.W + A.sub - 1) / A.sub, gh = (A.H + A.sub - 1) / A.sub;
    hipLaunchKernelGGL(reduce_slices, dim3((gw + 15) / 16, (gh + 15) / 16), dim3(kBlock), 0, stream, A,
                       (const float*)partial);
    return hipGetLastError();
}

hipError_t launch_upsample(const FrameArgs& A, hipStream_t stream) {
    hipLaunchKernelGGL(upsample_half, dim3((A.W + 15) / 16, (A.H + 15) / 16), dim3(kBlock), 0, stream, A);
    return hipGetLastError();
}

hipError_t launch_inject_bounce(const char* direct, int64_t direct_pitch, int direct_ch, int direct_f16,
                                const char* albedo, int64_t albedo_pitch, int albedo_ch, int albedo_f16,
                                const float* gi, int64_t gi_pitch, char* next, int64_t next_pitch, int next_ch,
                                int next_f16, int W, int H, float gain, hipStream_t stream) {
    const BounceArgs B{direct, albedo, gi, next, direct_pitch, albedo_pitch, gi_pitch, next_pitch,
                       W, H, direct_ch, albedo_ch, next_ch, direct_f16, albedo_f16, next_f16, gain};
    hipLaunchKernelGGL(inject_bounce, dim3((W + 63) / 64, (H + 3) / 4), dim3(kBlock), 0, stream, B);
    return hipGetLastError();
}

int slices_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gather_slices<32>, kBlock, 0) != hipSuccess || nb < 1)
        nb = 2;
    return nb;
}

int frame_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gather_frame<SSVB_HIT_ROUND, false, 0>, kBlock, 0) !=
            hipSuccess ||
        nb < 1)
        nb = 2;
    return nb;
}

hipError_t launch_debug_lattice(const FrameArgs& A, int32_t* out, hipStream_t stream) {
    hipLaunchKernelGGL(debug_lattice, grid16(A), dim3(kBlock), 0, stream, A, out);
    return hipGetLastError();
}

template <int CRIT>
static void launch_endpoints_fmt(const FrameArgs& A, float* out, hipStream_t stream) {
    switch (A.normal_f16) {
        case 0: hipLaunchKernelGGL((debug_endpoints<CRIT, 0>), grid16(A), dim3(kBlock), 0, stream, A, out); break;
        default: hipLaunchKernelGGL((debug_endpoints<CRIT, 1>), grid16(A), dim3(kBlock), 0, stream, A, out); break;
    }
}

hipError_t launch_debug_endpoints(const FrameArgs& A, float* out, hipStream_t stream) {
    if (A.criterion == SSVB_HIT_ROUND) launch_endpoints_fmt<SSVB_HIT_ROUND>(A, out, stream);
    else launch_endpoints_fmt<SSVB_HIT_PSEUDOCODE>(A, out, stream);
    return hipGetLastError();
}

}  // namespace ssvb
