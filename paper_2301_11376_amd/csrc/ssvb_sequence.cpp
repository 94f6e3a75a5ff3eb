// Frame sequences: multi-bounce feedback through a light buffer the sequence owns, and
// the noise seed advanced per frame (temporal jitter).  Section 4.3 injects a frame's
// indirect light into the light buffer of the next frame; Section 3.1 distributes the
// integral over time as well as space, and Section 4.1 times one slice per pixel turned
// from frame to frame.  A step is the elementwise injection (ssvb_inject_bounce) into the
// light buffer, the gather (ssvb_compute) on that light with seed + n, and a device copy
// of the frame's GI for the next step, all on the caller's stream.
#include <new>

#include "ssvb_host.h"

using namespace ssvb;

struct ssvb_sequence {
    ssvb_ctx* ctx = nullptr;
    int device = 0;
    int32_t W = 0, H = 0;
    ssvb_dtype light_dtype = SSVB_F32;
    void* light = nullptr;  // [H][W][3] light_dtype, dense
    float* gi = nullptr;    // [H][W][3] FP32: the GI of the last frame
    float* zero = nullptr;  // [H][W][3] FP32 zeros: the GI before frame 0
    int64_t frame = 0;
};

namespace {

struct DeviceScope {
    int prev = 0;
    bool switched = false;
    explicit DeviceScope(int device) {
        (void)hipGetDevice(&prev);
        if (prev != device) switched = hipSetDevice(device) == hipSuccess;
    }
    ~DeviceScope() {
        if (switched) (void)hipSetDevice(prev);
    }
};

ssvb_image light_image(const ssvb_sequence* q) {
    return ssvb_image{q->light, 0, q->light_dtype, 3};
}

void free_buffers(ssvb_sequence* q) {
    if (q->light) (void)hipFree(q->light);
    if (q->gi) (void)hipFree(q->gi);
    if (q->zero) (void)hipFree(q->zero);
    q->light = q->gi = q->zero = nullptr;
}

}  // namespace

extern "C" {

ssvb_status ssvb_sequence_create(ssvb_ctx* ctx, int32_t width, int32_t height, ssvb_dtype light_dtype,
                                 ssvb_sequence** out) {
    if (!out) return fail(SSVB_ERR_INVALID_ARG, "NULL output handle");
    *out = nullptr;
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    if (width < 1 || height < 1 || width > kMaxDim || height > kMaxDim)
        return fail(SSVB_ERR_INVALID_ARG, "sequence of %dx%d frames outside [1, %d]", width, height, kMaxDim);
    if (light_dtype != SSVB_F32 && light_dtype != SSVB_F16)
        return fail(SSVB_ERR_INVALID_ARG, "light dtype %d is not F32 or F16", light_dtype);
    ssvb_sequence* q = new (std::nothrow) ssvb_sequence();
    if (!q) return fail(SSVB_ERR_OUT_OF_MEMORY, "host allocation");
    q->ctx = ctx;
    q->device = ctx_device(ctx);
    q->W = width;
    q->H = height;
    q->light_dtype = light_dtype;
    const size_t px = (size_t)width * (size_t)height;
    DeviceScope dev(q->device);
    hipError_t e = hipMalloc(&q->light, px * 3 * (size_t)elem_size(light_dtype));
    if (e == hipSuccess) e = hipMalloc((void**)&q->gi, px * 12);
    if (e == hipSuccess) e = hipMalloc((void**)&q->zero, px * 12);
    if (e == hipSuccess) e = hipMemset(q->zero, 0, px * 12);
    if (e == hipSuccess) e = hipMemset(q->gi, 0, px * 12);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_buffers(q);
        delete q;
        return e == hipErrorOutOfMemory ? fail(SSVB_ERR_OUT_OF_MEMORY, "sequence buffers for %dx%d", width, height)
                                        : hip_fail(e, "sequence buffers");
    }
    *out = q;
    return SSVB_OK;
}

ssvb_status ssvb_sequence_step(ssvb_sequence* q, const ssvb_image* depth, const ssvb_image* normal,
                               const ssvb_image* direct, const ssvb_image* albedo, const ssvb_camera* camera,
                               const ssvb_params* params, float gain, const ssvb_outputs* out, void* hip_stream) {
    if (!q) return fail(SSVB_ERR_INVALID_ARG, "NULL sequence");
    if (!camera || !params) return fail(SSVB_ERR_INVALID_ARG, "NULL camera or params");
    if (camera->width != q->W || camera->height != q->H)
        return fail(SSVB_ERR_INVALID_ARG, "camera of %dx%d for a sequence of %dx%d frames", camera->width,
                    camera->height, q->W, q->H);
    // every argument is checked before the first launch
    const ssvb_image light = light_image(q);
    const float* prev = q->frame == 0 ? q->zero : q->gi;
    ssvb_status s = validate_bounce(q->W, q->H, direct, albedo, prev, 0, gain, &light);
    if (s) return s;
    ssvb_params p = *params;
    p.seed = (uint32_t)((uint64_t)params->seed + (uint64_t)q->frame);
    if ((s = ssvb_validate(depth, normal, &light, camera, &p, out))) return s;
    if ((s = ssvb_inject_bounce(q->ctx, q->W, q->H, direct, albedo, prev, 0, gain, &light, hip_stream))) return s;
    if ((s = ssvb_compute(q->ctx, depth, normal, &light, camera, &p, out, hip_stream))) return s;
    DeviceScope dev(q->device);
    const size_t row = (size_t)q->W * 12;
    const hipError_t e = hipMemcpy2DAsync(q->gi, row, out->gi, out->gi_pitch_bytes ? (size_t)out->gi_pitch_bytes : row,
                                          row, (size_t)q->H, hipMemcpyDeviceToDevice, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "copying the frame's GI");
    q->frame++;
    return SSVB_OK;
}

ssvb_status ssvb_sequence_reset(ssvb_sequence* q) {
    if (!q) return fail(SSVB_ERR_INVALID_ARG, "NULL sequence");
    q->frame = 0;
    return SSVB_OK;
}

ssvb_status ssvb_sequence_frame(ssvb_sequence* q, int64_t* frame) {
    if (!q || !frame) return fail(SSVB_ERR_INVALID_ARG, "NULL argument");
    *frame = q->frame;
    return SSVB_OK;
}

ssvb_status ssvb_sequence_copy_light(ssvb_sequence* q, void* dst, int64_t dst_pitch_bytes, void* hip_stream) {
    if (!q || !dst) return fail(SSVB_ERR_INVALID_ARG, "NULL argument");
    const size_t row = (size_t)q->W * 3 * (size_t)elem_size(q->light_dtype);
    if (dst_pitch_bytes != 0 && (dst_pitch_bytes < (int64_t)row))
        return fail(SSVB_ERR_INVALID_ARG, "pitch %lld bytes (row needs %zu)", (long long)dst_pitch_bytes, row);
    DeviceScope dev(q->device);
    const hipError_t e = hipMemcpy2DAsync(dst, dst_pitch_bytes ? (size_t)dst_pitch_bytes : row, q->light, row, row,
                                          (size_t)q->H, hipMemcpyDefault, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "copying the light buffer");
    return SSVB_OK;
}

ssvb_status ssvb_sequence_destroy(ssvb_sequence* q) {
    if (!q) return SSVB_OK;
    DeviceScope dev(q->device);
    free_buffers(q);
    delete q;
    return SSVB_OK;
}

}  // extern "C"
