// C ABI of the visibility-bitmask gather: argument validation, per-frame constants,
// context management and kernel launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "ssvb_denoise.h"
#include "ssvb_host.h"

using namespace ssvb;

constexpr int kBatchSlots = 2;  // descriptor slots of the batched path (double buffering)
constexpr int kRing = 32;       // queue-counter sets of single-frame launches that may be in flight
constexpr int kRingStride = 16; // uint32 per set (9 used)
constexpr int kMaxSliceChunk = 65536;  // tiles per chunk of the slice-major order

struct ssvb_ctx {
    int device = 0;
    int2 h_lut[kLutSize];
    FrameTables tab;  // device tables and launch shapes
    std::string tune_cache;
    // single-frame path: persistent grid and a ring of queue-counter sets, each guarded
    // by the event recorded after its last launch
    int frame_grid = 0;
    uint32_t* d_ring = nullptr;
    hipEvent_t ring_ev[kRing] = {};
    bool ring_pending[kRing] = {};
    uint64_t next_ring = 0;
    // slice-major order of ssvb_compute (0: off): chunk size in tiles, the partial-sum
    // buffer (grown on demand) and the event after its last use (slice-major launches on
    // any stream are ordered after the previous one, which shares the buffer)
    uint32_t slice_chunk = 0;
    int slices_grid = 0;
    int cus = 0;  // compute units of the device
    float* partial = nullptr;
    size_t partial_cap = 0;
    hipEvent_t partial_ev = nullptr;
    bool partial_pending = false;
    // batched path
    bool batch_ready = false;
    int batch_grid[2] = {0, 0};
    hipStream_t cap_stream = nullptr;
    BatchSlot slot[kBatchSlots];
    uint64_t next_slot = 0;
};

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace ssvb {

ssvb_status fail(ssvb_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

ssvb_status hip_fail(hipError_t e, const char* what) {
    return fail(SSVB_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const std::string& last_error() { return g_last_error; }

int ctx_device(const ssvb_ctx* ctx) { return ctx->device; }
const FrameTables* ctx_tables(const ssvb_ctx* ctx) { return &ctx->tab; }

}  // namespace ssvb

namespace {

bool finite(float v) { return isfinite(v) != 0; }

ssvb_status check_image(const ssvb_image* im, const char* name, int32_t W, int32_t H, bool is_depth) {
    if (!im) return fail(SSVB_ERR_INVALID_ARG, "%s: NULL image descriptor", name);
    if (is_depth) {
        if (im->dtype != SSVB_F32 || im->channels != 1)
            return fail(SSVB_ERR_INVALID_ARG, "%s: depth must be F32 with 1 channel", name);
    } else {
        if (im->dtype != SSVB_F32 && im->dtype != SSVB_F16)
            return fail(SSVB_ERR_INVALID_ARG, "%s: dtype %d is not F32 or F16", name, im->dtype);
        if (im->channels != 3 && im->channels != 4)
            return fail(SSVB_ERR_INVALID_ARG, "%s: %d channels (need 3 or 4)", name, im->channels);
    }
    if ((int64_t)W * H == 0) return SSVB_OK;
    if (!im->ptr) return fail(SSVB_ERR_INVALID_ARG, "%s: NULL pointer", name);
    const int64_t es = elem_size(im->dtype);
    if ((uintptr_t)im->ptr % es) return fail(SSVB_ERR_INVALID_ARG, "%s: pointer not aligned to %lld bytes", name, (long long)es);
    const int64_t row = (int64_t)W * im->channels * es;
    if (im->pitch_bytes != 0 && (im->pitch_bytes < row || im->pitch_bytes % es))
        return fail(SSVB_ERR_INVALID_ARG, "%s: pitch %lld bytes (row needs %lld, multiple of %lld)", name,
                    (long long)im->pitch_bytes, (long long)row, (long long)es);
    const int64_t pitch = im->pitch_bytes ? im->pitch_bytes : row;
    if (pitch * (H - 1) + row > ((int64_t)1 << 32))
        return fail(SSVB_ERR_INVALID_ARG, "%s: the image must span at most 4 GiB", name);
    return SSVB_OK;
}

ssvb_status check_out_pitch(int64_t pitch, int64_t row, const char* name) {
    if (pitch != 0 && (pitch < row || pitch % 4))
        return fail(SSVB_ERR_INVALID_ARG, "%s: pitch %lld bytes (row needs %lld, multiple of 4)", name,
                    (long long)pitch, (long long)row);
    return SSVB_OK;
}

// AO / GI / ambient image set of width W: present, 4-byte aligned, pitches that fit
ssvb_status check_signal(const ssvb_outputs* o, const char* name, int32_t W) {
    if (!o) return fail(SSVB_ERR_INVALID_ARG, "%s: NULL outputs", name);
    if (!o->ao || !o->gi || !o->ambient) return fail(SSVB_ERR_INVALID_ARG, "%s: ao, gi and ambient are required", name);
    if (o->masks) return fail(SSVB_ERR_INVALID_ARG, "%s: masks must be NULL", name);
    if (((uintptr_t)o->ao | (uintptr_t)o->gi | (uintptr_t)o->ambient) % 4)
        return fail(SSVB_ERR_INVALID_ARG, "%s: must be 4-byte aligned", name);
    ssvb_status s;
    if ((s = check_out_pitch(o->ao_pitch_bytes, (int64_t)W * 4, name))) return s;
    if ((s = check_out_pitch(o->gi_pitch_bytes, (int64_t)W * 12, name))) return s;
    if ((s = check_out_pitch(o->ambient_pitch_bytes, (int64_t)W * 12, name))) return s;
    return SSVB_OK;
}

// byte ranges [lo, hi) of the three images of a set
void signal_ranges(const ssvb_outputs* o, int32_t W, int32_t H, uintptr_t lo[3], uintptr_t hi[3]) {
    const int64_t row[3] = {(int64_t)W * 4, (int64_t)W * 12, (int64_t)W * 12};
    const int64_t pitch[3] = {o->ao_pitch_bytes ? o->ao_pitch_bytes : row[0],
                              o->gi_pitch_bytes ? o->gi_pitch_bytes : row[1],
                              o->ambient_pitch_bytes ? o->ambient_pitch_bytes : row[2]};
    const uintptr_t base[3] = {(uintptr_t)o->ao, (uintptr_t)o->gi, (uintptr_t)o->ambient};
    for (int i = 0; i < 3; ++i) {
        lo[i] = base[i];
        hi[i] = base[i] + (uintptr_t)(pitch[i] * (H - 1) + row[i]);
    }
}

bool sets_overlap(const ssvb_outputs* a, const ssvb_outputs* b, int32_t W, int32_t H) {
    uintptr_t alo[3], ahi[3], blo[3], bhi[3];
    signal_ranges(a, W, H, alo, ahi);
    signal_ranges(b, W, H, blo, bhi);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (alo[i] < bhi[j] && blo[j] < ahi[i]) return true;
    return false;
}

ssvb_status check_camera_params(const ssvb_camera* cam, const ssvb_params* p) {
    if (!cam) return fail(SSVB_ERR_INVALID_ARG, "NULL camera");
    if (!p) return fail(SSVB_ERR_INVALID_ARG, "NULL params");
    if (cam->width < 0 || cam->height < 0 || cam->width > kMaxDim || cam->height > kMaxDim)
        return fail(SSVB_ERR_INVALID_ARG, "image %dx%d outside [0, %d]", cam->width, cam->height, kMaxDim);
    if (!(finite(cam->fx) && cam->fx > 0 && finite(cam->fy) && cam->fy > 0))
        return fail(SSVB_ERR_INVALID_ARG, "focal lengths must be finite and > 0");
    if (!(finite(cam->cx) && finite(cam->cy))) return fail(SSVB_ERR_INVALID_ARG, "principal point not finite");
    for (int i = 0; i < 9; ++i)
        if (!finite(cam->view_to_world[i])) return fail(SSVB_ERR_INVALID_ARG, "view_to_world not finite");
    if (p->slices < 1 || p->slices > kMaxSlices)
        return fail(SSVB_ERR_INVALID_ARG, "slices %d outside [1, %d]", p->slices, kMaxSlices);
    if (p->steps < 1 || p->steps > kMaxSteps)
        return fail(SSVB_ERR_INVALID_ARG, "steps %d outside [1, %d]", p->steps, kMaxSteps);
    if (p->sectors <= 0) return fail(SSVB_ERR_INVALID_ARG, "sectors %d must be > 0", p->sectors);
    if (p->sectors != 32 && p->sectors != 128)
        return fail(SSVB_ERR_UNSUPPORTED, "sectors %d: the GPU path implements 32 and 128", p->sectors);
    const int na = p->ambient_samples;
    if (na < 1 || na > 32 || (p->sectors % na) != 0)
        return fail(SSVB_ERR_INVALID_ARG, "ambient_samples %d must be at most 32 and divide the sector count", na);
    if (!(finite(p->radius) && p->radius > 0)) return fail(SSVB_ERR_INVALID_ARG, "radius must be finite and > 0");
    if (!(p->thickness >= 0)) return fail(SSVB_ERR_INVALID_ARG, "thickness must be >= 0 (inf allowed)");
    if (!(finite(p->thickness_slope) && p->thickness_slope >= 0))
        return fail(SSVB_ERR_INVALID_ARG, "thickness_slope must be finite and >= 0");
    if (!(finite(p->max_radius_px) && p->max_radius_px >= 0))
        return fail(SSVB_ERR_INVALID_ARG, "max_radius_px must be finite and >= 0");
    if (p->min_step_q4 < 1 || p->min_step_q4 > 16)
        return fail(SSVB_ERR_INVALID_ARG, "min_step_q4 %d outside [1, 16]", p->min_step_q4);
    if (p->step_distribution != SSVB_STEPS_UNIFORM && p->step_distribution != SSVB_STEPS_QUADRATIC)
        return fail(SSVB_ERR_INVALID_ARG, "unknown step distribution %d", p->step_distribution);
    if (p->resolution != 1 && p->resolution != 2)
        return fail(SSVB_ERR_INVALID_ARG, "resolution divisor %d (need 1 or 2)", p->resolution);
    if (p->hit_criterion != SSVB_HIT_ROUND && p->hit_criterion != SSVB_HIT_PSEUDOCODE)
        return fail(SSVB_ERR_INVALID_ARG, "unknown hit criterion %d", p->hit_criterion);
    if (p->noise != SSVB_NOISE_HASH && p->noise != SSVB_NOISE_R2 && p->noise != SSVB_NOISE_FIXED)
        return fail(SSVB_ERR_INVALID_ARG, "unknown noise mode %d", p->noise);
    for (int i = 0; i < 27; ++i)
        if (!finite(p->ambient_sh[i])) return fail(SSVB_ERR_INVALID_ARG, "ambient_sh not finite");
    return SSVB_OK;
}

void r2_constants(uint32_t out[3]) {
    // Roberts' R2 sequence: g is the plastic number, the real root of g^3 = g + 1
    long double g = 1.3L;
    for (int i = 0; i < 100; ++i) g -= (g * g * g - g - 1.0L) / (3.0L * g * g - 1.0L);
    const long double two32 = 4294967296.0L;
    const long double phi = (1.0L + sqrtl(5.0L)) / 2.0L;
    out[0] = (uint32_t)llroundl(two32 / g);
    out[1] = (uint32_t)llroundl(two32 / (g * g));
    out[2] = (uint32_t)llroundl(two32 / phi);
}

}  // namespace

namespace ssvb {
// The context's tables, in FP64 on the host: the slice directions (Dx, Dy) =
// round(4096 (cos, sin)(pi k / 4096)), and cos / sin of h pi / 64 (h = -64..64) and of
// h pi / 256 (h = -256..256), the sector boundaries of the exact decisions.
void fill_tables(int2 lut[kLutSize], double2 half[129], double2 half128[513]) {
    for (int k = 0; k < kLutSize; ++k) {
        const double phi = M_PI * k / kLutSize;
        lut[k] = make_int2((int)floor(kLutOne * cos(phi) + 0.5), (int)floor(kLutOne * sin(phi) + 0.5));
    }
    for (int h = -64; h <= 64; ++h) half[h + 64] = make_double2(cos(M_PI * h / 64.0), sin(M_PI * h / 64.0));
    for (int h = -256; h <= 256; ++h) half128[h + 256] = make_double2(cos(M_PI * h / 256.0), sin(M_PI * h / 256.0));
}

// Apply a launch shape to a frame (clamped to valid values).
void set_launch(FrameArgs& A, LaunchShape L) {
    if (!(L.lp == 1 || L.lp == 2 || L.lp == 4 || L.lp == 8)) L.lp = 1;
    if (L.tile_w < 1 || L.tile_h < 1 || L.tile_w * L.tile_h * L.lp != 256) {
        L.tile_w = 32 / L.lp > 0 ? 32 / L.lp : 1;
        L.tile_h = 256 / L.lp / L.tile_w;
    }
    A.tile_w = L.tile_w;
    A.tile_h = L.tile_h;
    A.lp = L.lp;
    const int gw = (A.W + A.sub - 1) / A.sub, gh = (A.H + A.sub - 1) / A.sub;  // computed pixel grid
    A.tiles_x = (gw + A.tile_w - 1) / A.tile_w;
    A.tiles_y = (gh + A.tile_h - 1) / A.tile_h;
    A.strip = L.strip > 0 ? L.strip : 1;
    if (A.strip > A.tiles_x) A.strip = A.tiles_x > 0 ? A.tiles_x : 1;
}
}  // namespace ssvb

namespace ssvb {

// Fill the frame constants: FP64 derivation, one rounding to FP32.
void fill_frame(FrameArgs& A, const FrameTables* tab, const ssvb_image* depth, const ssvb_image* normal,
                const ssvb_image* radiance, const ssvb_camera* cam, const ssvb_params* p, const ssvb_outputs* out) {
    memset(&A, 0, sizeof A);
    const int W = cam->width, H = cam->height;
    A.W = W;
    A.H = H;
    A.depth = (const float*)depth->ptr;
    A.depth_pitch = depth->pitch_bytes ? depth->pitch_bytes : (int64_t)W * 4;
    if (normal) {
        A.normal = (const char*)normal->ptr;
        A.normal_ch = normal->channels;
        A.normal_f16 = normal->dtype == SSVB_F16;
        A.normal_pitch = normal->pitch_bytes ? normal->pitch_bytes : (int64_t)W * normal->channels * elem_size(normal->dtype);
    }
    if (radiance) {
        A.radiance = (const char*)radiance->ptr;
        A.radiance_ch = radiance->channels;
        A.radiance_f16 = radiance->dtype == SSVB_F16;
        A.radiance_pitch =
            radiance->pitch_bytes ? radiance->pitch_bytes : (int64_t)W * radiance->channels * elem_size(radiance->dtype);
    }
    if (out) {
        A.ao = out->ao;
        A.gi = out->gi;
        A.amb = out->ambient;
        A.masks = out->masks;
        A.ao_pitch = out->ao_pitch_bytes ? out->ao_pitch_bytes : (int64_t)W * 4;
        A.gi_pitch = out->gi_pitch_bytes ? out->gi_pitch_bytes : (int64_t)W * 12;
        A.amb_pitch = out->ambient_pitch_bytes ? out->ambient_pitch_bytes : (int64_t)W * 12;
        A.masks_pitch = out->masks_pitch_bytes ? out->masks_pitch_bytes : (int64_t)W * p->slices * (p->sectors / 32) * 4;
    }
    A.fx = cam->fx;
    A.fy = cam->fy;
    A.cx = cam->cx;
    A.cy = cam->cy;
    A.inv_fx = (float)(1.0 / cam->fx);
    A.inv_fy = (float)(1.0 / cam->fy);
    A.d3x = (float)(1.0 / (4096.0 * cam->fx));
    A.d3y = (float)(-1.0 / (4096.0 * cam->fy));
    for (int i = 0; i < 9; ++i) A.Rvw[i] = cam->view_to_world[i];
    A.nd = p->slices;
    A.ns = p->steps;
    A.na = p->ambient_samples;
    A.nb = p->sectors;
    A.criterion = p->hit_criterion;
    A.step_dist = p->step_distribution;
    A.sub = p->resolution == 2 ? 2 : 1;
    A.ns_recip = (uint32_t)(((uint64_t)1 << 32) / (uint64_t)(p->steps + 1));  // steps >= 1
    A.noise = p->noise;
    A.seed = p->seed;
    uint32_t r2[3];
    r2_constants(r2);
    A.r2a1 = r2[0];
    A.r2a2 = r2[1];
    A.r2a3 = r2[2];
    // step = r / (N_s + 1) with r = radius fy / z pixels; in 1/16 px: C / z
    A.c_step = (float)(16.0 * (double)p->radius * (double)cam->fy / (double)(p->steps + 1));
    const double rcap = p->max_radius_px > 0 ? fmin((double)p->max_radius_px, (double)kLatticeCapPx) : (double)kLatticeCapPx;
    A.q_min = p->min_step_q4;
    A.q_max = (int32_t)fmax((double)A.q_min, floor(16.0 * rcap / (double)(p->steps + 1)));
    A.q_max_f = (float)A.q_max;
    A.t0 = p->thickness;
    A.tk = p->thickness_slope;
    for (int i = 0; i < 27; ++i) A.sh[i] = p->ambient_sh[i];
    for (int k = 0; k < p->ambient_samples; ++k) {
        const double beta = -0.5 * M_PI + (k + 0.5) * M_PI / p->ambient_samples;
        A.amb_cb[k] = (float)cos(beta);
        A.amb_sb[k] = (float)sin(beta);
    }
    A.lut = tab ? tab->d_lut : nullptr;
    A.half_sector = tab ? (p->sectors == 128 ? tab->d_half128 : tab->d_half) : nullptr;
    LaunchShape shape{32, 8, 4, 1};
    if (tab) {
        if (tab->forced) {
            shape = tab->force;
        } else {
            const int fmt = (normal && normal->dtype == SSVB_F16 ? 1 : 0) | (radiance && radiance->dtype == SSVB_F16 ? 2 : 0);
            auto it = tab->tuned.find(ShapeKey{W, H, p->slices, p->steps, fmt});
            if (it != tab->tuned.end()) shape = it->second;
        }
    }
    set_launch(A, shape);
}

// Build one descriptor table: frame constants and the order of work (the order given;
// with work stealing inside each frame, sorting by cost measured no better).
void build_batch(const FrameTables* tab, BatchDesc* D, const ssvb_frame* frames, int n) {
    D->n_frames = n;
    for (int f = 0; f < n; ++f) {
        const ssvb_frame& F = frames[f];
        fill_frame(D->frames[f], tab, &F.depth, &F.normal, &F.radiance, &F.camera, &F.params, &F.out);
    }
    // per mask width: the frames in the given order, tile-count prefix sums, and runs of
    // equal sample cost (a tile costs tile pixels x slices x steps)
    for (int w = 0; w < 2; ++w) {
        int m = 0;
        uint32_t tiles = 0;
        double total = 0.0;
        D->prefix[w][0] = 0;
        for (int f = 0; f < n; ++f) {
            const FrameArgs& A = D->frames[f];
            if ((A.nb == 128) != (w == 1)) continue;
            D->plist[w][m] = f;
            tiles += (uint32_t)A.tiles_x * (uint32_t)A.tiles_y;
            D->prefix[w][++m] = tiles;
            total += (double)A.tiles_x * A.tiles_y * A.tile_w * A.tile_h * A.nd * A.ns;
        }
        D->pn[w] = m;
        D->split[w][0] = 0;
        int k = 1;
        double acc = 0.0;
        for (int j = 0; j < m && k < kXcds; ++j) {
            const FrameArgs& A = D->frames[D->plist[w][j]];
            const double per_tile = (double)A.tile_w * A.tile_h * A.nd * A.ns;
            const uint32_t nt = D->prefix[w][j + 1] - D->prefix[w][j];
            // the tiles of this frame at which the cumulative cost crosses k / kXcds of the total
            while (k < kXcds && acc + nt * per_tile >= total * k / kXcds) {
                const double need = total * k / kXcds - acc;
                uint32_t t = (uint32_t)ceil(need / per_tile);
                if (t > nt) t = nt;
                D->split[w][k++] = D->prefix[w][j] + t;
            }
            acc += nt * per_tile;
        }
        while (k <= kXcds) D->split[w][k++] = tiles;
    }
}

// Arguments of one denoising pass from `in` to `out` (validated inputs).
void fill_denoise(DenoiseArgs& D, const ssvb_image* depth, const ssvb_image* normal, const ssvb_camera* camera,
                  const ssvb_denoise_params* dp, const ssvb_outputs* in, const ssvb_outputs* out) {
    const int W = camera->width, H = camera->height;
    D = DenoiseArgs{};
    D.depth = (const float*)depth->ptr;
    D.depth_pitch = depth->pitch_bytes ? depth->pitch_bytes : (int64_t)W * 4;
    D.normal = (const char*)normal->ptr;
    D.normal_ch = normal->channels;
    D.normal_f16 = normal->dtype == SSVB_F16;
    D.normal_pitch = normal->pitch_bytes ? normal->pitch_bytes : (int64_t)W * normal->channels * elem_size(normal->dtype);
    D.W = W;
    D.H = H;
    D.g = dp->resolution;
    D.gw = (W + D.g - 1) / D.g;
    D.gh = (H + D.g - 1) / D.g;
    D.tiles_x = (D.gw + kDenoiseTile - 1) / kDenoiseTile;
    D.tiles = D.tiles_x * ((D.gh + kDenoiseTile - 1) / kDenoiseTile);
    D.cx = camera->cx;
    D.cy = camera->cy;
    D.inv_fx = (float)(1.0 / camera->fx);
    D.inv_fy = (float)(1.0 / camera->fy);
    D.inv_sigma = isinf(dp->plane_sigma) ? 0.0f : (float)(1.0 / (double)dp->plane_sigma);
    D.normal_power = dp->normal_power;
    D.in_ao = in->ao, D.in_gi = in->gi, D.in_amb = in->ambient;
    D.in_ao_pitch = in->ao_pitch_bytes ? in->ao_pitch_bytes : (int64_t)W * 4;
    D.in_gi_pitch = in->gi_pitch_bytes ? in->gi_pitch_bytes : (int64_t)W * 12;
    D.in_amb_pitch = in->ambient_pitch_bytes ? in->ambient_pitch_bytes : (int64_t)W * 12;
    D.out_ao = out->ao, D.out_gi = out->gi, D.out_amb = out->ambient;
    D.out_ao_pitch = out->ao_pitch_bytes ? out->ao_pitch_bytes : (int64_t)W * 4;
    D.out_gi_pitch = out->gi_pitch_bytes ? out->gi_pitch_bytes : (int64_t)W * 12;
    D.out_amb_pitch = out->ambient_pitch_bytes ? out->ambient_pitch_bytes : (int64_t)W * 12;
}

// Frame constants of the half-resolution fill of the signal set `out` (the upsampler reads
// depth and writes the uncomputed pixels in place).
void fill_upsample(FrameArgs& A, const ssvb_image* depth, const ssvb_camera* camera, const ssvb_outputs* out) {
    const int W = camera->width, H = camera->height;
    memset(&A, 0, sizeof A);
    A.depth = (const float*)depth->ptr;
    A.depth_pitch = depth->pitch_bytes ? depth->pitch_bytes : (int64_t)W * 4;
    A.W = W;
    A.H = H;
    A.ao = out->ao, A.gi = out->gi, A.amb = out->ambient;
    A.ao_pitch = out->ao_pitch_bytes ? out->ao_pitch_bytes : (int64_t)W * 4;
    A.gi_pitch = out->gi_pitch_bytes ? out->gi_pitch_bytes : (int64_t)W * 12;
    A.amb_pitch = out->ambient_pitch_bytes ? out->ambient_pitch_bytes : (int64_t)W * 12;
}

hipError_t batch_grid_size(int device, int grid[2]) {
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return e;
    for (int i = 0; i < 2; ++i) {
        const int per_cu = batch_blocks_per_cu(i ? 128 : 32);
        grid[i] = ((prop.multiProcessorCount * per_cu + kXcds - 1) / kXcds) * kXcds;
    }
    return hipSuccess;
}

hipError_t init_slot(BatchSlot& s) {
    hipError_t e = hipHostMalloc((void**)&s.h_desc, sizeof(BatchDesc), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&s.d_desc, sizeof(BatchDesc));
    if (e == hipSuccess) e = hipMalloc((void**)&s.d_queues, kBatchQueues * sizeof(uint32_t));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e == hipSuccess) memset(s.h_desc, 0, sizeof(BatchDesc));
    return e;
}

hipError_t slot_graph(BatchSlot& s, int kinds, const int grid[2], hipStream_t cap_stream, hipGraphExec_t* exec) {
    if (!s.exec[kinds]) {
        hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        const hipError_t ce = enqueue_batch(s.d_desc, s.h_desc, s.d_queues, grid, kinds, cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cap_stream, &g);
        if (ce != hipSuccess) e = ce;
        if (e == hipSuccess) e = hipGraphInstantiate(&s.exec[kinds], g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            s.exec[kinds] = nullptr;
            return e;
        }
        s.graph[kinds] = g;
    }
    *exec = s.exec[kinds];
    return hipSuccess;
}

void free_slot(BatchSlot& s) {
    for (int i = 0; i < kBatchKinds; ++i) {
        if (s.exec[i]) (void)hipGraphExecDestroy(s.exec[i]);
        if (s.graph[i]) (void)hipGraphDestroy(s.graph[i]);
    }
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.d_queues) (void)hipFree(s.d_queues);
    if (s.d_desc) (void)hipFree(s.d_desc);
    if (s.h_desc) (void)hipHostFree(s.h_desc);
    s = BatchSlot{};
}

}  // namespace ssvb

namespace {

bool valid_shape(const ssvb_launch* L) {
    if (!L) return false;
    const int lp = L->lanes_per_pixel;
    return (lp == 1 || lp == 2 || lp == 4 || lp == 8) && L->tile_w > 0 && L->tile_h > 0 &&
           L->tile_w * L->tile_h * lp == 256 && L->strip > 0;
}

void load_tune_cache(ssvb_ctx* ctx) {
    const char* path = getenv("SSVB_TUNE_CACHE");
    if (!path || !*path) return;
    ctx->tune_cache = path;
    FILE* f = fopen(path, "r");
    if (!f) return;
    int W, H, nd, ns, fmt, tw, th, st, lp;
    float ms;
    while (fscanf(f, "%d %d %d %d %d %d %d %d %d %f", &W, &H, &nd, &ns, &fmt, &tw, &th, &st, &lp, &ms) == 10) {
        ssvb_launch L{tw, th, st, lp};
        if (valid_shape(&L)) ctx->tab.tuned[ShapeKey{W, H, nd, ns, fmt}] = LaunchShape{tw, th, st, lp};
    }
    fclose(f);
}

ssvb_status init_batch(ssvb_ctx* ctx) {
    if (ctx->batch_ready) return SSVB_OK;
    hipError_t e = batch_grid_size(ctx->device, ctx->batch_grid);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
    for (int k = 0; k < kBatchSlots && e == hipSuccess; ++k) e = init_slot(ctx->slot[k]);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(SSVB_ERR_OUT_OF_MEMORY, "batch buffers")
                                                          : hip_fail(e, "batch set-up");
    ctx->batch_ready = true;
    return SSVB_OK;
}

void free_batch(ssvb_ctx* ctx) {
    for (int k = 0; k < kBatchSlots; ++k) free_slot(ctx->slot[k]);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    ctx->cap_stream = nullptr;
    ctx->batch_ready = false;
}

}  // namespace

extern "C" {

const char* ssvb_status_string(ssvb_status s) {
    switch (s) {
        case SSVB_OK: return "SSVB_OK";
        case SSVB_ERR_INVALID_ARG: return "SSVB_ERR_INVALID_ARG";
        case SSVB_ERR_UNSUPPORTED: return "SSVB_ERR_UNSUPPORTED";
        case SSVB_ERR_OUT_OF_MEMORY: return "SSVB_ERR_OUT_OF_MEMORY";
        case SSVB_ERR_DEVICE: return "SSVB_ERR_DEVICE";
        case SSVB_ERR_BUSY: return "SSVB_ERR_BUSY";
        case SSVB_ERR_TIMEOUT: return "SSVB_ERR_TIMEOUT";
        case SSVB_ERR_NOT_FOUND: return "SSVB_ERR_NOT_FOUND";
    }
    return "SSVB_ERR_UNKNOWN";
}

const char* ssvb_last_error(void) { return g_last_error.c_str(); }

void ssvb_default_params(ssvb_params* p) {
    if (!p) return;
    memset(p, 0, sizeof *p);
    p->slices = 4;
    p->steps = 16;
    p->sectors = 32;
    p->ambient_samples = 4;
    p->radius = 1.0f;
    p->thickness = 0.5f;
    p->thickness_slope = 0.0f;
    p->max_radius_px = 0.0f;
    p->min_step_q4 = 16;
    p->step_distribution = SSVB_STEPS_UNIFORM;
    p->resolution = 1;
    p->hit_criterion = SSVB_HIT_ROUND;
    p->noise = SSVB_NOISE_HASH;
    p->seed = 0;
}

ssvb_status ssvb_create(int32_t device, ssvb_ctx** out) {
    if (!out) return fail(SSVB_ERR_INVALID_ARG, "NULL output handle");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(SSVB_ERR_INVALID_ARG, "device %d of %d", device, count);
    ssvb_ctx* ctx = new (std::nothrow) ssvb_ctx();
    if (!ctx) return fail(SSVB_ERR_OUT_OF_MEMORY, "host allocation");
    ctx->device = device;
    double2 half[129], half128[513];
    fill_tables(ctx->h_lut, half, half128);
    int prev = 0;
    (void)hipGetDevice(&prev);
    if ((e = hipSetDevice(device)) != hipSuccess) {
        delete ctx;
        return hip_fail(e, "hipSetDevice");
    }
    load_tune_cache(ctx);
    e = hipMalloc((void**)&ctx->tab.d_lut, sizeof ctx->h_lut);
    if (e == hipSuccess) e = hipMemcpy(ctx->tab.d_lut, ctx->h_lut, sizeof ctx->h_lut, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->tab.d_half, sizeof half);
    if (e == hipSuccess) e = hipMemcpy(ctx->tab.d_half, half, sizeof half, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->tab.d_half128, sizeof half128);
    if (e == hipSuccess) e = hipMemcpy(ctx->tab.d_half128, half128, sizeof half128, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_ring, kRing * kRingStride * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(ctx->d_ring, 0, kRing * kRingStride * sizeof(uint32_t));
    for (int k = 0; k < kRing && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ctx->ring_ev[k], hipEventDisableTiming);
    if (e == hipSuccess) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, device);
        ctx->frame_grid = prop.multiProcessorCount * frame_blocks_per_cu();
        ctx->cus = prop.multiProcessorCount;
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        if (ctx->tab.d_lut) (void)hipFree(ctx->tab.d_lut);
        if (ctx->tab.d_half) (void)hipFree(ctx->tab.d_half);
        if (ctx->tab.d_half128) (void)hipFree(ctx->tab.d_half128);
        if (ctx->d_ring) (void)hipFree(ctx->d_ring);
        for (int k = 0; k < kRing; ++k)
            if (ctx->ring_ev[k]) (void)hipEventDestroy(ctx->ring_ev[k]);
        delete ctx;
        return e == hipErrorOutOfMemory ? fail(SSVB_ERR_OUT_OF_MEMORY, "direction table") : hip_fail(e, "direction table");
    }
    *out = ctx;
    return SSVB_OK;
}

ssvb_status ssvb_destroy(ssvb_ctx* ctx) {
    if (!ctx) return SSVB_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    free_batch(ctx);
    if (ctx->tab.d_lut) (void)hipFree(ctx->tab.d_lut);
    if (ctx->tab.d_half) (void)hipFree(ctx->tab.d_half);
    if (ctx->tab.d_half128) (void)hipFree(ctx->tab.d_half128);
    if (ctx->d_ring) (void)hipFree(ctx->d_ring);
    for (int k = 0; k < kRing; ++k)
        if (ctx->ring_ev[k]) (void)hipEventDestroy(ctx->ring_ev[k]);
    if (ctx->partial) (void)hipFree(ctx->partial);
    if (ctx->partial_ev) (void)hipEventDestroy(ctx->partial_ev);
    (void)hipSetDevice(prev);
    delete ctx;
    return SSVB_OK;
}

ssvb_status ssvb_validate(const ssvb_image* depth, const ssvb_image* normal, const ssvb_image* radiance,
                          const ssvb_camera* camera, const ssvb_params* params, const ssvb_outputs* out) {
    ssvb_status s = check_camera_params(camera, params);
    if (s) return s;
    const int W = camera->width, H = camera->height;
    if ((s = check_image(depth, "depth", W, H, true))) return s;
    if ((s = check_image(normal, "normal", W, H, false))) return s;
    if ((s = check_image(radiance, "radiance", W, H, false))) return s;
    if (!out) return fail(SSVB_ERR_INVALID_ARG, "NULL outputs");
    if ((int64_t)W * H == 0) return SSVB_OK;
    if (!out->ao || !out->gi || !out->ambient) return fail(SSVB_ERR_INVALID_ARG, "ao, gi and ambient are required");
    if (((uintptr_t)out->ao | (uintptr_t)out->gi | (uintptr_t)out->ambient | (uintptr_t)out->masks) % 4)
        return fail(SSVB_ERR_INVALID_ARG, "outputs must be 4-byte aligned");
    if ((s = check_out_pitch(out->ao_pitch_bytes, (int64_t)W * 4, "ao"))) return s;
    if ((s = check_out_pitch(out->gi_pitch_bytes, (int64_t)W * 12, "gi"))) return s;
    if ((s = check_out_pitch(out->ambient_pitch_bytes, (int64_t)W * 12, "ambient"))) return s;
    if (out->masks && (s = check_out_pitch(out->masks_pitch_bytes,
                                           (int64_t)W * params->slices * (params->sectors / 32) * 4, "masks")))
        return s;
    if (out->masks && params->resolution == 2)
        return fail(SSVB_ERR_INVALID_ARG, "slice masks exist only for computed pixels: not with half resolution");
    return SSVB_OK;
}

}  // extern "C"

namespace {

// Makes the context's device current for the lifetime of the guard (the test hooks below
// run on whatever device the caller left current otherwise).
struct DeviceGuard {
    int prev = 0;
    bool switched = false;
    explicit DeviceGuard(int device) {
        (void)hipGetDevice(&prev);
        if (prev != device) switched = hipSetDevice(device) == hipSuccess;
    }
    ~DeviceGuard() {
        if (switched) (void)hipSetDevice(prev);
    }
};

// One frame as a persistent single-frame launch (and the half-resolution fill) on
// `stream`.  A counter set of the ring is reused only once its previous launch has
// completed (blocks the host only with kRing launches of this context still in flight).
hipError_t launch_single(ssvb_ctx* ctx, const FrameArgs& A, hipStream_t stream) {
    const int r = (int)(ctx->next_ring++ % kRing);
    hipError_t e = hipSuccess;
    if (ctx->ring_pending[r]) e = hipEventSynchronize(ctx->ring_ev[r]);
    if (e == hipSuccess) e = launch_plain(A, ctx->d_ring + r * kRingStride, ctx->frame_grid, stream);
    if (e == hipSuccess && A.sub == 2) e = launch_upsample(A, stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ring_ev[r], stream);
    if (e == hipSuccess) ctx->ring_pending[r] = true;
    return e;
}

// The same frame in slice-major order (ctx->slice_chunk > 0): one lane per pixel, the
// per-slice gather into the context's partial buffer (grown when the frame needs more; the
// old buffer is freed once its last launch has completed), the reduction, the
// half-resolution fill.  Ordered after the previous slice-major launch of the context.
hipError_t launch_single_slices(ssvb_ctx* ctx, FrameArgs A, hipStream_t stream) {
    // set up on first use, so that a context that never turns the order on is unchanged
    if (!ctx->partial_ev) {
        const hipError_t c = hipEventCreateWithFlags(&ctx->partial_ev, hipEventDisableTiming);
        if (c != hipSuccess) {
            ctx->partial_ev = nullptr;
            return c;
        }
        ctx->slices_grid = ctx->cus * slices_blocks_per_cu();
    }
    if (A.lp > 1) set_launch(A, LaunchShape{A.tile_w * A.lp, A.tile_h, A.strip, 1});
    const size_t gw = (size_t)(A.W + A.sub - 1) / A.sub, gh = (size_t)(A.H + A.sub - 1) / A.sub;
    const size_t bytes = gw * gh * (size_t)A.nd * kPartialFloats * sizeof(float);
    hipError_t e = hipSuccess;
    if (bytes > ctx->partial_cap) {
        if (ctx->partial_pending) e = hipEventSynchronize(ctx->partial_ev);
        if (e == hipSuccess && ctx->partial) e = hipFree(ctx->partial);
        ctx->partial = nullptr;
        ctx->partial_cap = 0;
        if (e == hipSuccess) e = hipMalloc((void**)&ctx->partial, bytes);
        if (e != hipSuccess) return e;
        ctx->partial_cap = bytes;
    }
    if (ctx->partial_pending) e = hipStreamWaitEvent(stream, ctx->partial_ev, 0);
    const int r = (int)(ctx->next_ring++ % kRing);
    if (e == hipSuccess && ctx->ring_pending[r]) e = hipEventSynchronize(ctx->ring_ev[r]);
    if (e == hipSuccess)
        e = launch_slices(A, ctx->d_ring + r * kRingStride, ctx->slices_grid, ctx->partial, ctx->slice_chunk, stream);
    if (e == hipSuccess && A.sub == 2) e = launch_upsample(A, stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ring_ev[r], stream);
    if (e == hipSuccess) ctx->ring_pending[r] = true;
    if (e == hipSuccess) e = hipEventRecord(ctx->partial_ev, stream);
    if (e == hipSuccess) ctx->partial_pending = true;
    return e;
}

}  // namespace

extern "C" {

ssvb_status ssvb_compute(ssvb_ctx* ctx, const ssvb_image* depth, const ssvb_image* normal, const ssvb_image* radiance,
                         const ssvb_camera* camera, const ssvb_params* params, const ssvb_outputs* out,
                         void* hip_stream) {
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    ssvb_status s = ssvb_validate(depth, normal, radiance, camera, params, out);
    if (s) return s;
    if ((int64_t)camera->width * camera->height == 0) return SSVB_OK;
    FrameArgs A;
    fill_frame(A, &ctx->tab, depth, normal, radiance, camera, params, out);
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
    const hipError_t e = ctx->slice_chunk ? launch_single_slices(ctx, A, (hipStream_t)hip_stream)
                                          : launch_single(ctx, A, (hipStream_t)hip_stream);
    if (prev != ctx->device) (void)hipSetDevice(prev);
    if (e == hipErrorOutOfMemory && ctx->slice_chunk)
        return fail(SSVB_ERR_OUT_OF_MEMORY, "partial sums of the slice-major order");
    if (e != hipSuccess) return hip_fail(e, "gather launch");
    return SSVB_OK;
}

ssvb_status ssvb_set_slice_order(ssvb_ctx* ctx, int32_t chunk_tiles) {
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    if (chunk_tiles < 0 || chunk_tiles > kMaxSliceChunk)
        return fail(SSVB_ERR_INVALID_ARG, "chunk of %d tiles outside [0, %d]", chunk_tiles, kMaxSliceChunk);
    ctx->slice_chunk = (uint32_t)chunk_tiles;
    return SSVB_OK;
}

ssvb_status ssvb_compute_batch(ssvb_ctx* ctx, const ssvb_frame* frames, int32_t n, void* hip_stream) {
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    if (n < 0 || (n > 0 && !frames)) return fail(SSVB_ERR_INVALID_ARG, "bad frame array");
    for (int f = 0; f < n; ++f) {
        const ssvb_frame& F = frames[f];
        ssvb_status s = ssvb_validate(&F.depth, &F.normal, &F.radiance, &F.camera, &F.params, &F.out);
        if (s) return fail(s, "frame %d: %s", f, last_error().c_str());
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
    ssvb_status st = init_batch(ctx);
    hipStream_t stream = (hipStream_t)hip_stream;
    for (int f0 = 0; st == SSVB_OK && f0 < n; f0 += kMaxBatch) {
        // frames with no pixels launch nothing; frames of more than kPackTiles tiles are
        // single-frame launches (each fills the GPU by itself, and a launch of its own
        // keeps its L2 locality); the others are packed into one replay of the batch graph
        std::vector<ssvb_frame> chunk;
        std::vector<FrameArgs> large;
        int kinds = 0;
        for (int f = f0; f < std::min(n, f0 + kMaxBatch); ++f) {
            const ssvb_frame& F = frames[f];
            if ((int64_t)F.camera.width * F.camera.height == 0) continue;
            FrameArgs A;
            fill_frame(A, &ctx->tab, &F.depth, &F.normal, &F.radiance, &F.camera, &F.params, &F.out);
            if ((uint32_t)A.tiles_x * (uint32_t)A.tiles_y > kPackTiles) {
                large.push_back(A);
                continue;
            }
            chunk.push_back(F);
            kinds |= (F.params.sectors == 128 ? kBatch128 : kBatch32) | (F.params.resolution == 2 ? kBatchHalf : 0);
        }
        for (size_t j = 0; j < large.size() && st == SSVB_OK; ++j) {
            const hipError_t e = launch_single(ctx, large[j], stream);
            if (e != hipSuccess) st = hip_fail(e, "gather launch");
        }
        if (chunk.empty() || st != SSVB_OK) continue;
        BatchSlot& S = ctx->slot[ctx->next_slot++ % kBatchSlots];
        hipGraphExec_t exec = nullptr;
        hipError_t e = slot_graph(S, kinds, ctx->batch_grid, ctx->cap_stream, &exec);
        if (e == hipSuccess && S.pending) e = hipEventSynchronize(S.done);  // the slot's last upload is done
        if (e == hipSuccess) {
            build_batch(&ctx->tab, S.h_desc, chunk.data(), (int)chunk.size());
            e = hipGraphLaunch(exec, stream);
        }
        if (e == hipSuccess) e = hipEventRecord(S.done, stream);
        if (e != hipSuccess) st = hip_fail(e, "batch launch");
        else S.pending = true;
    }
    if (prev != ctx->device) (void)hipSetDevice(prev);
    return st;
}

ssvb_status ssvb_set_launch(ssvb_ctx* ctx, const ssvb_launch* shape) {
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    if (!shape) {
        ctx->tab.forced = false;
        return SSVB_OK;
    }
    if (!valid_shape(shape)) return fail(SSVB_ERR_INVALID_ARG, "launch shape needs tile_w*tile_h*lanes = 256, lanes 1/2/4/8, strip > 0");
    ctx->tab.forced = true;
    ctx->tab.force = LaunchShape{shape->tile_w, shape->tile_h, shape->strip, shape->lanes_per_pixel};
    return SSVB_OK;
}

ssvb_status ssvb_get_launch(ssvb_ctx* ctx, const ssvb_camera* camera, const ssvb_params* params, int32_t fp16_mask,
                            ssvb_launch* out) {
    if (!ctx || !camera || !params || !out) return fail(SSVB_ERR_INVALID_ARG, "NULL argument");
    ssvb_image n{nullptr, 0, (fp16_mask & 1) ? SSVB_F16 : SSVB_F32, 3};
    ssvb_image r{nullptr, 0, (fp16_mask & 2) ? SSVB_F16 : SSVB_F32, 3};
    ssvb_image d{nullptr, 0, SSVB_F32, 1};
    FrameArgs A;
    fill_frame(A, &ctx->tab, &d, &n, &r, camera, params, nullptr);
    *out = ssvb_launch{A.tile_w, A.tile_h, A.strip, A.lp};
    return SSVB_OK;
}

ssvb_status ssvb_autotune(ssvb_ctx* ctx, const ssvb_frame* frame, void* hip_stream, ssvb_launch* best, float* best_ms) {
    if (!ctx || !frame) return fail(SSVB_ERR_INVALID_ARG, "NULL argument");
    const ssvb_frame& F = *frame;
    ssvb_status s = ssvb_validate(&F.depth, &F.normal, &F.radiance, &F.camera, &F.params, &F.out);
    if (s) return s;
    if ((int64_t)F.camera.width * F.camera.height == 0) return fail(SSVB_ERR_INVALID_ARG, "empty frame");
    static const int kTiles[][3] = {{32, 8, 1}, {16, 16, 1}, {64, 4, 1}, {8, 32, 1}, {16, 8, 2}, {8, 16, 2},
                                    {32, 4, 2}, {8, 8, 4},   {16, 4, 4}, {8, 4, 8},  {4, 8, 8}};
    static const int kStrips[] = {1, 2, 4, 8};
    hipStream_t stream = (hipStream_t)hip_stream;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
    const bool was_forced = ctx->tab.forced;
    const LaunchShape was = ctx->tab.force;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best_t = 1e30f;
    LaunchShape best_s{32, 8, 4, 1};
    for (const auto& tl : kTiles) {
        for (int st : kStrips) {
            if (e != hipSuccess) break;
            ctx->tab.forced = true;
            ctx->tab.force = LaunchShape{tl[0], tl[1], st, tl[2]};
            float times[3];
            for (int rep = -1; rep < 3 && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, stream);
                if (e == hipSuccess && (s = ssvb_compute(ctx, &F.depth, &F.normal, &F.radiance, &F.camera, &F.params,
                                                         &F.out, hip_stream)) != SSVB_OK)
                    e = hipErrorUnknown;
                if (e == hipSuccess) e = hipEventRecord(e1, stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess && rep >= 0) e = hipEventElapsedTime(&times[rep], e0, e1);
            }
            if (e != hipSuccess) break;
            std::sort(times, times + 3);
            if (times[1] < best_t) {
                best_t = times[1];
                best_s = ctx->tab.force;
            }
        }
    }
    ctx->tab.forced = was_forced;
    ctx->tab.force = was;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (prev != ctx->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return s != SSVB_OK ? s : hip_fail(e, "autotune");
    const int fmt = (F.normal.dtype == SSVB_F16 ? 1 : 0) | (F.radiance.dtype == SSVB_F16 ? 2 : 0);
    ctx->tab.tuned[ShapeKey{F.camera.width, F.camera.height, F.params.slices, F.params.steps, fmt}] = best_s;
    if (!ctx->tune_cache.empty()) {
        if (FILE* f = fopen(ctx->tune_cache.c_str(), "a")) {
            fprintf(f, "%d %d %d %d %d %d %d %d %d %.4f\n", F.camera.width, F.camera.height, F.params.slices,
                    F.params.steps, fmt, best_s.tile_w, best_s.tile_h, best_s.strip, best_s.lp, best_t);
            fclose(f);
        }
    }
    if (best) *best = ssvb_launch{best_s.tile_w, best_s.tile_h, best_s.strip, best_s.lp};
    if (best_ms) *best_ms = best_t;
    return SSVB_OK;
}

}  // extern "C"

namespace ssvb {
// The checks of ssvb_inject_bounce, before anything is launched.
ssvb_status validate_bounce(int32_t width, int32_t height, const ssvb_image* direct, const ssvb_image* albedo,
                            const float* gi, int64_t gi_pitch_bytes, float gain, const ssvb_image* next) {
    if (width < 0 || height < 0 || width > kMaxDim || height > kMaxDim)
        return fail(SSVB_ERR_INVALID_ARG, "image %dx%d outside [0, %d]", width, height, kMaxDim);
    if (!(finite(gain) && gain >= 0.0f)) return fail(SSVB_ERR_INVALID_ARG, "gain must be finite and >= 0");
    ssvb_status s;
    if ((s = check_image(direct, "direct", width, height, false))) return s;
    if ((s = check_image(albedo, "albedo", width, height, false))) return s;
    if ((s = check_image(next, "next", width, height, false))) return s;
    if (next->channels != direct->channels && !(next->channels == 3 && direct->channels == 4))
        return fail(SSVB_ERR_INVALID_ARG, "next has %d channels, direct %d", next->channels, direct->channels);
    if ((int64_t)width * height == 0) return SSVB_OK;
    if (!gi || (uintptr_t)gi % 4) return fail(SSVB_ERR_INVALID_ARG, "gi: NULL or misaligned");
    if ((s = check_out_pitch(gi_pitch_bytes, (int64_t)width * 12, "gi"))) return s;
    return SSVB_OK;
}
}  // namespace ssvb

extern "C" {

ssvb_status ssvb_inject_bounce(ssvb_ctx* ctx, int32_t width, int32_t height, const ssvb_image* direct,
                               const ssvb_image* albedo, const float* gi, int64_t gi_pitch_bytes, float gain,
                               const ssvb_image* next, void* hip_stream) {
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    ssvb_status s = validate_bounce(width, height, direct, albedo, gi, gi_pitch_bytes, gain, next);
    if (s) return s;
    if ((int64_t)width * height == 0) return SSVB_OK;
    auto pitch = [&](const ssvb_image* im) {
        return im->pitch_bytes ? im->pitch_bytes : (int64_t)width * im->channels * elem_size(im->dtype);
    };
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
    const hipError_t e = launch_inject_bounce(
        (const char*)direct->ptr, pitch(direct), direct->channels, direct->dtype == SSVB_F16, (const char*)albedo->ptr,
        pitch(albedo), albedo->channels, albedo->dtype == SSVB_F16, gi,
        gi_pitch_bytes ? gi_pitch_bytes : (int64_t)width * 12, (char*)next->ptr, pitch(next), next->channels,
        next->dtype == SSVB_F16, width, height, gain, (hipStream_t)hip_stream);
    if (prev != ctx->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "bounce launch");
    return SSVB_OK;
}

void ssvb_default_denoise_params(ssvb_denoise_params* p) {
    if (!p) return;
    p->passes = 2;
    p->normal_power = 16;
    p->plane_sigma = 0.05f;
    p->resolution = 1;
}

ssvb_status ssvb_denoise(ssvb_ctx* ctx, const ssvb_image* depth, const ssvb_image* normal, const ssvb_camera* camera,
                         const ssvb_outputs* in, const ssvb_outputs* tmp, const ssvb_outputs* out,
                         const ssvb_denoise_params* dp, void* hip_stream) {
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    if (!camera) return fail(SSVB_ERR_INVALID_ARG, "NULL camera");
    if (!dp) return fail(SSVB_ERR_INVALID_ARG, "NULL denoise parameters");
    const int W = camera->width, H = camera->height;
    if (W < 0 || H < 0 || W > kMaxDim || H > kMaxDim)
        return fail(SSVB_ERR_INVALID_ARG, "image %dx%d outside [0, %d]", W, H, kMaxDim);
    if (!(finite(camera->fx) && camera->fx > 0 && finite(camera->fy) && camera->fy > 0))
        return fail(SSVB_ERR_INVALID_ARG, "focal lengths must be finite and > 0");
    if (!(finite(camera->cx) && finite(camera->cy))) return fail(SSVB_ERR_INVALID_ARG, "principal point not finite");
    if (dp->passes < 1 || dp->passes > 3) return fail(SSVB_ERR_INVALID_ARG, "passes %d outside [1, 3]", dp->passes);
    if (dp->normal_power < 0 || dp->normal_power > 128)
        return fail(SSVB_ERR_INVALID_ARG, "normal_power %d outside [0, 128]", dp->normal_power);
    if (!(dp->plane_sigma > 0)) return fail(SSVB_ERR_INVALID_ARG, "plane_sigma must be > 0 (inf allowed)");
    if (dp->resolution != 1 && dp->resolution != 2)
        return fail(SSVB_ERR_INVALID_ARG, "resolution divisor %d (need 1 or 2)", dp->resolution);
    ssvb_status s;
    if ((s = check_image(depth, "depth", W, H, true))) return s;
    if ((s = check_image(normal, "normal", W, H, false))) return s;
    if ((s = check_signal(in, "in", W))) return s;
    if ((s = check_signal(out, "out", W))) return s;
    if (dp->passes > 1 && (s = check_signal(tmp, "tmp", W))) return s;
    if ((int64_t)W * H == 0) return SSVB_OK;
    if (sets_overlap(in, out, W, H)) return fail(SSVB_ERR_INVALID_ARG, "in and out overlap");
    if (dp->passes > 1 && (sets_overlap(in, tmp, W, H) || sets_overlap(tmp, out, W, H)))
        return fail(SSVB_ERR_INVALID_ARG, "tmp overlaps in or out");

    DenoiseArgs D;
    hipStream_t stream = (hipStream_t)hip_stream;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
    hipError_t e = hipSuccess;
    const ssvb_outputs* src = in;
    for (int i = 0; i < dp->passes && e == hipSuccess; ++i) {
        // the passes alternate so that the last one writes `out`
        const ssvb_outputs* dst = ((dp->passes - 1 - i) % 2 == 0) ? out : tmp;
        fill_denoise(D, depth, normal, camera, dp, src, dst);
        e = launch_denoise(D, i, stream);
        src = dst;
    }
    if (e == hipSuccess && dp->resolution == 2) {
        FrameArgs A;
        fill_upsample(A, depth, camera, out);
        e = launch_upsample(A, stream);
    }
    if (prev != ctx->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "denoise launch");
    return SSVB_OK;
}

ssvb_status ssvb_debug_lattice(ssvb_ctx* ctx, const ssvb_image* depth, const ssvb_camera* camera,
                               const ssvb_params* params, int32_t* xy_out, void* hip_stream) {
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    ssvb_status s = check_camera_params(camera, params);
    if (s) return s;
    if ((s = check_image(depth, "depth", camera->width, camera->height, true))) return s;
    if ((int64_t)camera->width * camera->height == 0) return SSVB_OK;
    if (!xy_out) return fail(SSVB_ERR_INVALID_ARG, "NULL lattice output");
    FrameArgs A;
    fill_frame(A, &ctx->tab, depth, nullptr, nullptr, camera, params, nullptr);
    DeviceGuard g(ctx->device);
    hipError_t e = launch_debug_lattice(A, xy_out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "lattice launch");
    return SSVB_OK;
}

ssvb_status ssvb_debug_endpoints(ssvb_ctx* ctx, const ssvb_image* depth, const ssvb_image* normal,
                                 const ssvb_camera* camera, const ssvb_params* params, float* ep_out,
                                 void* hip_stream) {
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    ssvb_status s = check_camera_params(camera, params);
    if (s) return s;
    if (params->sectors != 32) return fail(SSVB_ERR_UNSUPPORTED, "the endpoint hook reports 32-sector coordinates");
    const int W = camera->width, H = camera->height;
    if ((s = check_image(depth, "depth", W, H, true))) return s;
    if ((s = check_image(normal, "normal", W, H, false))) return s;
    if ((int64_t)W * H == 0) return SSVB_OK;
    if (!ep_out) return fail(SSVB_ERR_INVALID_ARG, "NULL endpoint output");
    FrameArgs A;
    fill_frame(A, &ctx->tab, depth, normal, nullptr, camera, params, nullptr);
    hipStream_t st = (hipStream_t)hip_stream;
    DeviceGuard g(ctx->device);
    const size_t bytes = (size_t)W * H * params->slices * 2 * params->steps * 2 * sizeof(float);
    hipError_t e = hipMemsetAsync(ep_out, 0xFF, bytes, st);  // all-ones = NaN for skipped samples
    if (e == hipSuccess) e = launch_debug_endpoints(A, ep_out, st);
    if (e != hipSuccess) return hip_fail(e, "endpoint launch");
    return SSVB_OK;
}

ssvb_status ssvb_debug_direction_table(ssvb_ctx* ctx, int32_t* host_out) {
    if (!ctx || !host_out) return fail(SSVB_ERR_INVALID_ARG, "NULL argument");
    int2 tmp[kLutSize];
    DeviceGuard g(ctx->device);
    hipError_t e = hipMemcpy(tmp, ctx->tab.d_lut, sizeof tmp, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "direction table copy");
    for (int k = 0; k < kLutSize; ++k) {
        host_out[2 * k] = tmp[k].x;
        host_out[2 * k + 1] = tmp[k].y;
    }
    return SSVB_OK;
}

void ssvb_debug_noise_constants(uint32_t* host_out) {
    if (host_out) r2_constants(host_out);
}

}  // extern "C"
