/*
 * ssvb.h - C ABI of the screen-space visibility-bitmask gather on AMD Instinct MI355X
 * (gfx950).
 *
 * The operation is the per-pixel gather of Therrien, Levesque and Gilet, "Screen Space
 * Indirect Lighting with Visibility Bitmask" (arXiv 2301.11376): Algorithm 1 (ambient
 * occlusion and indirect diffuse light from an N_b-sector visibility bitmask per
 * hemisphere slice, Section 3.1 and Section 3.3) plus directionally occluded ambient
 * light (Section 3.2).  Inputs are the single-layer G-buffer the paper assumes: linear
 * view depth, view-space normals and an HDR buffer of direct light (Section 4.3).
 *
 * Conventions shared by every entry point
 *  - Images are row-major, interleaved channels (HWC).  Pixel (x, y) has its centre at
 *    (x + 0.5, y + 0.5); image y grows downward.  View space: x right, y up, camera
 *    looking down -z.  The view ray through screen point (X, Y) is
 *    ((X - cx)/fx, -(Y - cy)/fy, -1); a point at linear view depth z on it is z * ray.
 *  - Depth <= 0 or non-finite marks background.  A background pixel outputs AO = 1,
 *    GI = 0, ambient = 0 and empty masks; background samples are skipped.
 *  - Normals must be unit view-space vectors (used as stored).  Radiance is RGB.
 *  - Every image and output pointer is DEVICE memory owned by the caller.  The library
 *    never frees, retains or writes through caller memory after the call's work on the
 *    caller's stream has completed.
 *  - Calls that launch work are asynchronous on the caller's HIP stream (NULL = the
 *    legacy default stream).  Errors are returned, never thrown; arguments are validated
 *    before anything is launched, so an error leaves the outputs untouched.
 *  - A context may be used from one host thread at a time.
 */
#ifndef SSVB_H
#define SSVB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSVB_OK = 0,
    SSVB_ERR_INVALID_ARG = 1,   /* a pointer, size, pitch or parameter is out of range */
    SSVB_ERR_UNSUPPORTED = 2,   /* valid request the GPU path does not implement (e.g. N_b 64) */
    SSVB_ERR_OUT_OF_MEMORY = 3, /* device allocation failed, or a request exceeds a budget */
    SSVB_ERR_DEVICE = 4,        /* a HIP runtime call failed */
    SSVB_ERR_BUSY = 5,          /* the resource is in use (server slot or queue full) */
    SSVB_ERR_TIMEOUT = 6,       /* a wait exceeded its deadline */
    SSVB_ERR_NOT_FOUND = 7      /* unknown ticket or handle */
} ssvb_status;

typedef enum { SSVB_F32 = 0, SSVB_F16 = 1 } ssvb_dtype;

/* Hit criterion (Section 3.1).  ROUND sets a sector iff its centre lies in the sample's
 * angular interval (a sector counts once half of it is covered).  PSEUDOCODE takes the floor of the start
 * and the ceiling of the width, as Algorithm 1 prints it. */
typedef enum { SSVB_HIT_ROUND = 0, SSVB_HIT_PSEUDOCODE = 1 } ssvb_hit_criterion;

/* Per-pixel slice rotation and per-slice step jitter (Algorithm 1: directions with a
 * random offset; Section 4.3: jitter along the sampling direction).
 *  HASH : rho = pcg(x + pcg(y + pcg(seed))) >> 16, the PCG hash of Jarzynski and Olano
 *         (JCGT 2020);
 *  R2   : rho = (x a1 + y a2 + seed a3 mod 2^32) >> 16, Roberts' R2 dither
 *         (a1 = round(2^32/g), a2 = round(2^32/g^2), g the plastic number,
 *          a3 = round(2^32/phi));
 *  FIXED: rho = 0, no jitter.
 * In HASH and R2 the jitter of slice i is pcg(x + pcg(y + pcg(seed + 1 + i))) >> 24. */
typedef enum { SSVB_NOISE_HASH = 0, SSVB_NOISE_R2 = 1, SSVB_NOISE_FIXED = 2 } ssvb_noise;

/* Placement of the N_s steps along each side of a slice.  UNIFORM (Algorithm 1): step j
 * (0-based) at (j + 1 + xi) / (N_s + 1) of the reach.  QUADRATIC (Section 4.3 distributes
 * samples more densely near the pixel; the curve is this library's choice): at
 * ((j + 1 + xi) / (N_s + 1))^2 of the reach.  xi is the slice's jitter; the reach is
 * q (N_s + 1) sixteenths of a pixel in both, q the pixel's step length. */
typedef enum { SSVB_STEPS_UNIFORM = 0, SSVB_STEPS_QUADRATIC = 1 } ssvb_step_distribution;

/* One image.  ptr: device pointer aligned to its element size.  pitch_bytes: bytes
 * between rows, 0 = dense (width * channels * element size).  dtype: ssvb_dtype.
 * channels: 1 for depth (F32 only), 3 or 4 for normals and radiance (the fourth
 * channel is ignored).  Every image (pitch * (height - 1) + row bytes) must span at
 * most 4 GiB. */
typedef struct {
    const void* ptr;
    int64_t pitch_bytes;
    int32_t dtype;
    int32_t channels;
} ssvb_image;

/* Pinhole camera.  width, height in [0, 16384].  fx, fy > 0 in pixels.
 * view_to_world: row-major rotation, world_dir = M * view_dir (used for the ambient
 * probe, which lives in world space). */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float view_to_world[9];
} ssvb_camera;

/* Sampling parameters (Algorithm 1; Sections 3.1-3.3).
 *  slices           N_d, hemisphere slices per pixel, 1..64
 *  steps            N_s, depth samples per side of each slice, 1..1024
 *  sectors          N_b, bits of the visibility mask: 32 or 128 (Section 4.1 reports 32
 *                   as enough and 128 as 5-10 % slower)
 *  ambient_samples  N_a, ambient subregions per slice, at most 32, divides N_b
 *  radius           world-space radius of the screen-aligned hemisphere, > 0
 *  thickness        t0 >= 0 (+inf allowed: GTAO without falloff, Section 3.1)
 *  thickness_slope  k >= 0: each pixel uses t = t0 + k * depth (Section 3.1)
 *  max_radius_px    0, or a cap in pixels on the projected radius (hard cap 16383)
 *  min_step_q4      shortest step in 1/16 pixel, 1..16 (16 keeps samples off the
 *                   centre pixel)
 *  step_distribution  ssvb_step_distribution
 *  resolution       1: every pixel is gathered; 2: half resolution (Section 4.3): only
 *                   pixels with both coordinates even are gathered (reading the full
 *                   G-buffer), every other pixel averages its 1, 2 or 4 nearest gathered
 *                   pixels with weights bilinear x (1e-3 + exp(-((z - z_n)/(0.05 z))^2))
 *                   (background neighbours excluded; none left: AO 1, GI 0, ambient 0).
 *                   No slice masks.
 *  hit_criterion    ssvb_hit_criterion
 *  noise, seed      ssvb_noise and its 32-bit seed
 *  ambient_sh       L2 real spherical-harmonic probe, world space, [9][3]
 *                   coefficient-major RGB (the ambient light source of Section 3.2) */
typedef struct {
    int32_t slices, steps, sectors, ambient_samples;
    float radius, thickness, thickness_slope, max_radius_px;
    int32_t min_step_q4;
    int32_t step_distribution;
    int32_t resolution;
    int32_t hit_criterion;
    int32_t noise;
    uint32_t seed;
    float ambient_sh[27];
} ssvb_params;

/* Outputs, FP32, device memory.  ao [H][W]; gi and ambient [H][W][3]; masks, if not
 * NULL, [H][W][N_d][N_b / 32] uint32 with sector k in bit k % 32 of word k / 32 (sector k
 * spans angles [-pi/2 + k pi/N_b, -pi/2 + (k+1) pi/N_b] from the projected normal, k
 * increasing toward the slice direction).  Pitches in bytes, 0 = dense.  AO is
 * visibility (1 = open). */
typedef struct {
    float* ao;
    float* gi;
    float* ambient;
    uint32_t* masks;
    int64_t ao_pitch_bytes, gi_pitch_bytes, ambient_pitch_bytes, masks_pitch_bytes;
} ssvb_outputs;

/* One frame of a batch: inputs, camera, parameters and outputs (as for ssvb_compute). */
typedef struct {
    ssvb_image depth, normal, radiance;
    ssvb_camera camera;
    ssvb_params params;
    ssvb_outputs out;
} ssvb_frame;

/* Launch shape of the gather: workgroups of tile_w x tile_h pixels with lanes_per_pixel
 * lanes each (tile_w * tile_h * lanes_per_pixel = 256; lanes_per_pixel in {1, 2, 4, 8}
 * splits a pixel's slices over adjacent lanes), tiles walked in vertical strips of
 * `strip` tiles.  Shapes change speed only, never results beyond FP32 summation order. */
typedef struct {
    int32_t tile_w, tile_h, strip, lanes_per_pixel;
} ssvb_launch;

typedef struct ssvb_ctx ssvb_ctx;

/* Human-readable name of a status code.  Never NULL. */
const char* ssvb_status_string(ssvb_status s);

/* Detail of the most recent error raised on the calling host thread ("" if none). */
const char* ssvb_last_error(void);

/* Fill *p with the defaults: 4 slices, 16 steps, 32 sectors, 4 ambient samples,
 * radius 1, thickness 0.5, slope 0, no pixel cap, min step 16, uniform steps, full
 * resolution, ROUND, HASH, seed 0, zero ambient probe. */
void ssvb_default_params(ssvb_params* p);

/* Create a context on HIP device `device`: uploads the slice-direction table.  The
 * context owns only its own device buffers.  *out receives the handle. */
ssvb_status ssvb_create(int32_t device, ssvb_ctx** out);

/* Destroy a context created by ssvb_create (NULL is ignored).  Waits for nothing: the
 * caller must have synchronised the streams it used with this context. */
ssvb_status ssvb_destroy(ssvb_ctx* ctx);

/* Host-only argument check of one frame, exactly as ssvb_compute performs it; touches
 * no device and needs no context. */
ssvb_status ssvb_validate(const ssvb_image* depth, const ssvb_image* normal,
                          const ssvb_image* radiance, const ssvb_camera* camera,
                          const ssvb_params* params, const ssvb_outputs* out);

/* The visibility-bitmask gather of one frame (Algorithm 1 with the ambient term of
 * Section 3.2): writes AO, GI (RGB indirect diffuse) and ambient (RGB), each divided by
 * N_d, and optionally the N_d slice masks.  Asynchronous on `hip_stream`: one persistent
 * kernel whose workgroups take the frame's tiles from per-XCD work queues.  The context
 * keeps 32 sets of queue counters; a call blocks the host only if the launch that last
 * used its set (32 calls earlier) has not yet finished. */
ssvb_status ssvb_compute(ssvb_ctx* ctx, const ssvb_image* depth, const ssvb_image* normal,
                         const ssvb_image* radiance, const ssvb_camera* camera,
                         const ssvb_params* params, const ssvb_outputs* out, void* hip_stream);

/* Many frames of mixed size, slice/step counts, criteria, mask widths, resolutions and
 * element types, asynchronous on `hip_stream`.  Frames of at most 8,192 tiles (1920x1080
 * at the default launch shape) go into one replay of a captured HIP graph (descriptor
 * upload, queue reset, a persistent kernel per mask width present, then the
 * half-resolution fill if any frame asks for it) with their tiles packed into one list
 * cut into equal-cost runs, one per XCD; larger frames each get the persistent
 * single-frame launch of ssvb_compute (each fills the GPU by itself; always in the
 * default work order, see ssvb_set_slice_order).  Each frame's outputs equal, bit for
 * bit, what ssvb_compute writes for it with the same launch shape and the default work
 * order.  The first batch with a new set of frame kinds (mask widths, half resolution)
 * captures that set's graph on the calling thread: meanwhile no other thread may
 * synchronise the whole device.  Frames are processed in chunks of 64.  The library keeps
 * two descriptor slots and the 32 counter sets of ssvb_compute, so a call may block until
 * the batch submitted two chunks earlier, or the launch 32 large frames earlier, has
 * finished.  Returns SSVB_ERR_INVALID_ARG naming the first invalid frame. */
ssvb_status ssvb_compute_batch(ssvb_ctx* ctx, const ssvb_frame* frames, int32_t n, void* hip_stream);

/* Force one launch shape for every later frame of this context (NULL: back to the
 * autotuned shape of the frame's class, else the default 32 x 8, strip 4, 1 lane). */
ssvb_status ssvb_set_launch(ssvb_ctx* ctx, const ssvb_launch* shape);

/* Work order of this context's later ssvb_compute calls, frame sequences included (not
 * batches or servers).
 * chunk_tiles 0 (the default): each workgroup runs every slice of its tile.  chunk_tiles
 * C in 1..65536: slice-major order, for cache locality (a pixel's slices turn by its own
 * random offset, so one slice of many pixels samples one wedge of directions rather than
 * the whole disc, Algorithm 1): the work items of each die's run of tiles are (tile,
 * slice) pairs, taken for slice 0 of C tiles, then slice 1 of the same C tiles, and so
 * on; one lane per pixel (a shape with more lanes keeps its pixel count with one lane);
 * each item writes its slice's sums (32 bytes per computed pixel and slice) to a buffer
 * the context allocates and grows on demand (freed with the context; growing it waits
 * for the context's previous slice-major launch), and a second kernel adds the slices in
 * order.  AO and the masks equal the default order's bit for bit; GI and ambient sum the
 * same terms grouped by slice (FP32 rounding).  Slice-major launches of one context are
 * ordered one after another on the device whatever their streams, since they share the
 * buffer.  SSVB_ERR_INVALID_ARG for C outside [0, 65536]; ssvb_compute returns
 * SSVB_ERR_OUT_OF_MEMORY when the buffer cannot grow. */
ssvb_status ssvb_set_slice_order(ssvb_ctx* ctx, int32_t chunk_tiles);

/* The launch shape ssvb_compute would use for this camera / parameter / element-type
 * class (fp16_mask: bit 0 normals FP16, bit 1 radiance FP16). */
ssvb_status ssvb_get_launch(ssvb_ctx* ctx, const ssvb_camera* camera, const ssvb_params* params,
                            int32_t fp16_mask, ssvb_launch* out);

/* Time candidate launch shapes on `frame` (its outputs are overwritten; synchronises
 * `hip_stream`), remember the fastest for the frame's class (width, height, slices,
 * steps, element types) and return it with its time in ms.  If the environment variable
 * SSVB_TUNE_CACHE names a file, tuned shapes are loaded from it by ssvb_create and
 * appended to it here. */
ssvb_status ssvb_autotune(ssvb_ctx* ctx, const ssvb_frame* frame, void* hip_stream, ssvb_launch* best,
                          float* best_ms);

/* Multi-bounce indirect light (Section 4.3: the indirect light is injected into the light
 * buffer used by the next frame, its intensity scaled down): writes, per pixel and RGB
 * channel, next = direct + gain * albedo * gi.  direct and albedo: images of width x height
 * (F32 or F16, 3 or 4 channels); gi: FP32 [height][width][3] as ssvb_compute writes it,
 * row pitch gi_pitch_bytes (0 = dense); next: an image of the same channel count as
 * direct, or of 3 channels (F32 or F16; F16 rounds to nearest even); a fourth channel of
 * next is copied from direct.  next may be direct itself (each element is read before it is written).
 * gain finite and >= 0 (>= 1 lets repeated bounces grow without bound).  Asynchronous
 * on hip_stream; validated before anything is launched. */
ssvb_status ssvb_inject_bounce(ssvb_ctx* ctx, int32_t width, int32_t height, const ssvb_image* direct,
                               const ssvb_image* albedo, const float* gi, int64_t gi_pitch_bytes, float gain,
                               const ssvb_image* next, void* hip_stream);

/* A sequence of frames of one size with multi-bounce feedback and temporal jitter.
 * Section 4.3 injects a frame's indirect light into the light buffer the next frame uses;
 * Section 3.1 distributes the integral over time as well as space, and Section 4.1 times
 * one slice per pixel turned from frame to frame.  The sequence owns, in device memory
 * allocated here (the only allocation; steps allocate nothing), its light buffer
 * (width x height x 3 of light_dtype, F32 or F16), the FP32 GI of the last frame and a
 * zeroed FP32 GI image that stands for the frame before frame 0 (width x height x 3 each):
 * 36 (F32 light) or 30 (F16) bytes per pixel.  The frame counter starts at 0.  Errors:
 * SSVB_ERR_INVALID_ARG (size outside [1, 16384], dtype), SSVB_ERR_OUT_OF_MEMORY,
 * SSVB_ERR_DEVICE. */
typedef struct ssvb_sequence ssvb_sequence;
ssvb_status ssvb_sequence_create(ssvb_ctx* ctx, int32_t width, int32_t height, ssvb_dtype light_dtype,
                                 ssvb_sequence** out);

/* Frame n of the sequence (n = the frame counter), asynchronous on hip_stream:
 *   1. light = direct + gain * albedo * GI of frame n - 1 (nothing before frame 0), written
 *      to the sequence's light buffer as ssvb_inject_bounce writes it (FP32 arithmetic);
 *   2. the gather of ssvb_compute on (depth, normal, light) with params->seed + n (mod
 *      2^32), so the slice rotations and step jitters change from frame to frame;
 *   3. out receives AO, GI, ambient (and the slice masks if out->masks is set) as
 *      ssvb_compute writes them, and the GI is copied to the sequence for frame n + 1.
 * direct and albedo: images of the sequence's size (F32 or F16, 3 or 4 channels); depth,
 * normal, camera, params and out as for ssvb_compute, the camera of the sequence's size.
 * gain finite and >= 0.  Everything is validated before anything is launched; the frame
 * counter advances only when the step was enqueued.  Steps of one sequence must be
 * ordered on the device (one stream, or the caller orders them); steps of different
 * sequences are independent.  A step uses the sequence's context, so the context's rule
 * holds: one host thread at a time. */
ssvb_status ssvb_sequence_step(ssvb_sequence* seq, const ssvb_image* depth, const ssvb_image* normal,
                               const ssvb_image* direct, const ssvb_image* albedo, const ssvb_camera* camera,
                               const ssvb_params* params, float gain, const ssvb_outputs* out, void* hip_stream);

/* Set the frame counter to 0: the next step has no feedback and uses params->seed. */
ssvb_status ssvb_sequence_reset(ssvb_sequence* seq);

/* The frame counter (frames stepped since creation or the last reset). */
ssvb_status ssvb_sequence_frame(ssvb_sequence* seq, int64_t* frame);

/* Copy the light buffer of the last step (width x height x 3 of the light type, dense
 * rows) to `dst` (device or host memory, rows of dst_pitch_bytes, 0 = dense), ordered on
 * hip_stream after that step. */
ssvb_status ssvb_sequence_copy_light(ssvb_sequence* seq, void* dst, int64_t dst_pitch_bytes, void* hip_stream);

/* Free the sequence's buffers (after its work on the device has finished).  NULL is
 * ignored. */
ssvb_status ssvb_sequence_destroy(ssvb_sequence* seq);

/* Parameters of ssvb_denoise.
 *  passes        1..3: pass i averages over 5 x 5 taps 2^i cells apart
 *  normal_power  k in 0..128: a tap weighs max(0, n_p . n_q)^k by its normal
 *  plane_sigma   > 0 (+inf: no plane term): a tap weighs exp(-d^2) by its plane
 *                distance d = n_p . (P_q - P_p) / (plane_sigma z_p), P the view-space
 *                position z r(x, y) of the pixel centre
 *  resolution    1: every pixel; 2: the outputs of a half-resolution ssvb_compute (the
 *                filter runs on the pixels with both coordinates even, then the
 *                half-resolution fill of ssvb_params.resolution refills the others) */
typedef struct {
    int32_t passes;
    int32_t normal_power;
    float plane_sigma;
    int32_t resolution;
} ssvb_denoise_params;

/* passes 2, normal_power 16, plane_sigma 0.05, resolution 1 */
void ssvb_default_denoise_params(ssvb_denoise_params* p);

/* Edge-aware a-trous denoising of AO, GI and ambient (Section 4.1 and Table 2 time a
 * denoising pass after the gather without describing it; this filter is the library's
 * own): each pass replaces every foreground pixel's seven values by the average over its
 * taps with weights h_a h_b exp(-d^2) max(0, n_p . n_q)^k, h = (1, 4, 6, 4, 1) / 16,
 * the pixel's own weight h_0^2; taps off the image or on background (depth <= 0 or not
 * finite) are left out; background pixels keep their input.  depth and normal as for
 * ssvb_compute (the normal renormalised); camera: width, height, fx, fy, cx, cy.  `in`,
 * `tmp` and `out` hold AO, GI and ambient as ssvb_compute writes them (masks must be
 * NULL); the passes alternate between tmp and out so that the last one writes out; tmp
 * is needed for 2 or 3 passes (NULL members allowed for 1).  The three sets must not
 * overlap.  `in` is not modified.  Asynchronous on hip_stream; validated before anything
 * is launched. */
ssvb_status ssvb_denoise(ssvb_ctx* ctx, const ssvb_image* depth, const ssvb_image* normal,
                         const ssvb_camera* camera, const ssvb_outputs* in, const ssvb_outputs* tmp,
                         const ssvb_outputs* out, const ssvb_denoise_params* params, void* hip_stream);

/* ---------------------------------------------------------------------------------
 * Request loop.  A server owns an arena of device memory (its HBM budget) and a
 * scheduler thread.  Submitted frames wait in arrival order until their footprint fits
 * in the arena:
 *     W * H * (4 + normal bytes/px + radiance bytes/px + 28), each part 256-aligned
 * (depth FP32, the normal and radiance buffers as given, AO + GI + ambient FP32).
 * An admitted frame holds that much of the arena until it has finished: its buffers that
 * are in host memory are copied into it on a copy stream (results copied back), buffers
 * already in this device's memory are read and written in place.  As soon as one of the
 * server's compute streams is idle, every admitted frame not yet started (at most 64)
 * forms one round on it: its small frames (at most 8,192 tiles, 1920x1080 at the default
 * shape) in one launch of the batch kernel with their tiles packed into one list, then
 * its larger frames as persistent single-frame launches back to back.  A request is done
 * as soon as its own part of the round (the packed frames, or its single-frame launch)
 * and its result copies have finished.  Frames that arrive while a round is on the device join the next
 * one, and rounds on different streams overlap.  Every mode of ssvb_compute is served
 * (128 sectors, half resolution; not slice masks).  Each frame's results are those
 * ssvb_compute writes for it with the launch shape of its class.
 * Ownership: the frame's input and output pointers (device memory, or host memory that
 * should be pinned for the copies to be asynchronous) must stay valid, and the inputs
 * unchanged, until the request has finished; the outputs are written before `done` is
 * reported.  A server keeps the context's device tables and a snapshot of its launch
 * shapes: the context must outlive it.  Server calls are thread-safe; one thread must
 * not release a ticket another thread is waiting on.
 * --------------------------------------------------------------------------------- */
typedef struct ssvb_server ssvb_server;

/* Counters of a server since its creation (current values where noted). */
typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t rounds;                  /* rounds started */
    uint64_t frames_in_rounds;        /* frames over all rounds */
    uint64_t admitted_while_running;  /* frames admitted while a round was on the device */
    uint64_t arena_bytes, arena_in_use, arena_peak; /* in_use: current */
    int32_t queued;                   /* current: waiting for memory */
    int32_t resident;                 /* current: in the arena */
    int32_t running_rounds;           /* current */
    int32_t max_running_rounds;       /* most rounds on the device at once */
    int32_t max_round_frames;         /* largest round */
    int32_t reserved;
} ssvb_server_counters;

/* Create a server on ctx's device with an arena of hbm_budget_bytes (allocated here;
 * SSVB_ERR_OUT_OF_MEMORY if it cannot be) and `streams` compute streams (1..8, 0 = 1).
 * With one stream a round starts when the previous one has finished (the gap is the
 * scheduler's turnaround, tens of microseconds); with more, rounds run concurrently, which
 * on MI355X measured slower (every round's persistent kernels want all CUs): 0.96 of the
 * one-stream throughput with two streams, 0.87 with three or four. */
ssvb_status ssvb_server_create(ssvb_ctx* ctx, uint64_t hbm_budget_bytes, int32_t streams, ssvb_server** out);

/* Queue one frame (validated as by ssvb_compute; masks must be NULL) and return its
 * ticket.  Never blocks on the device.  hip_stream is the stream on which the caller last
 * wrote or read the frame's buffers (inputs and outputs; NULL is the null stream): an
 * event is recorded on it here, and every copy and kernel of the server that touches this
 * request's buffers waits for that event, so the request sees all work the caller
 * enqueued on that stream before this call, with no host synchronisation.  Work on other
 * streams must be ordered before this call by the caller.  The buffers must stay alive
 * and must not be written by the caller until the request has finished.
 * SSVB_ERR_OUT_OF_MEMORY if its footprint exceeds the whole arena; SSVB_ERR_BUSY if 2^20
 * tickets are unreleased or the server is being destroyed; SSVB_ERR_DEVICE after a device
 * error stopped the server, or if the event cannot be recorded on hip_stream.  A frame
 * with no pixels finishes at once. */
ssvb_status ssvb_server_submit(ssvb_server* server, const ssvb_frame* frame, void* hip_stream, uint64_t* ticket);

/* *done = 1 once the request's outputs are in the caller's buffers; *latency_ms (may be
 * NULL) is then the time from submission to completion.  SSVB_ERR_NOT_FOUND for an
 * unknown or released ticket; SSVB_ERR_DEVICE (with *done = 1) if it failed. */
ssvb_status ssvb_server_poll(ssvb_server* server, uint64_t ticket, int32_t* done, double* latency_ms);

/* Block until the request finishes or timeout_ms passes (negative: no limit); returns
 * SSVB_ERR_TIMEOUT if it has not finished by then. */
ssvb_status ssvb_server_wait(ssvb_server* server, uint64_t ticket, double timeout_ms, double* latency_ms);

/* Forget a finished request (SSVB_ERR_BUSY if it has not finished). */
ssvb_status ssvb_server_release(ssvb_server* server, uint64_t ticket);

/* Copy the server's counters. */
ssvb_status ssvb_server_stats(ssvb_server* server, ssvb_server_counters* out);

/* Stop the server: requests not yet started are dropped, rounds on the device are waited
 * for, then the arena, streams and thread are freed.  NULL is ignored. */
ssvb_status ssvb_server_destroy(ssvb_server* server);

/* Test hook: the integer step lattice of ssvb_compute.  xy_out (device, int32) receives,
 * for every pixel, slice, side (+ then -) and step, the sampled texel (X, Y), laid out
 * [H][W][N_d][2][N_s][2] densely.  Same validation of depth/camera/params. */
ssvb_status ssvb_debug_lattice(ssvb_ctx* ctx, const ssvb_image* depth, const ssvb_camera* camera,
                               const ssvb_params* params, int32_t* xy_out, void* hip_stream);

/* Test hook: the FP32 sector-boundary arguments of every sample, as ssvb_compute
 * computes them before its FP64 re-decision near a boundary.  ep_out (device, float)
 * receives [H][W][N_d][2][N_s][2]: for ROUND the two values whose floor gives the
 * sample's sectors [a, b) (32 u + 1/2 at each end of its angular interval, u in [0, 1]
 * across the hemisphere), for PSEUDOCODE the floor argument of the start and the ceiling
 * argument of the width.  Skipped samples are NaN. */
ssvb_status ssvb_debug_endpoints(ssvb_ctx* ctx, const ssvb_image* depth, const ssvb_image* normal,
                                 const ssvb_camera* camera, const ssvb_params* params, float* ep_out,
                                 void* hip_stream);

/* Test hook: copy the 4096-entry slice-direction table (Dx, Dy pairs, fixed point
 * 1 = 4096, direction pi k / 4096) to host memory `host_out` (8192 int32). */
ssvb_status ssvb_debug_direction_table(ssvb_ctx* ctx, int32_t* host_out);

/* Test hook: the R2 constants a1, a2, a3 (host memory, 3 uint32).  Host only. */
void ssvb_debug_noise_constants(uint32_t* host_out);

#ifdef __cplusplus
}
#endif

#endif /* SSVB_H */
