// Host-side pieces shared by the C ABI (ssvb_api.cpp) and the request loop
// (ssvb_server.cpp): frame and denoiser constants, launch-shape tables, batch descriptor
// slots, launchers and error reporting.
#ifndef SSVB_HOST_H
#define SSVB_HOST_H

#include <map>
#include <string>
#include <tuple>

#include "ssvb_denoise.h"
#include "ssvb_internal.h"

namespace ssvb {

// frame class for tuned launch shapes: width, height, slices, steps, FP16 mask
using ShapeKey = std::tuple<int, int, int, int, int>;

// What the frame constants need from a context: device tables and launch shapes.
struct FrameTables {
    int2* d_lut = nullptr;      // slice directions
    double2* d_half = nullptr;     // cos, sin of h pi / 64, h = -64..64 (32 sectors)
    double2* d_half128 = nullptr;  // cos, sin of h pi / 256, h = -256..256 (128 sectors)
    bool forced = false;
    LaunchShape force{32, 8, 4, 1};
    std::map<ShapeKey, LaunchShape> tuned;
};

// One descriptor slot of the batched path: pinned + device descriptor table, the queue
// heads (one per frame and XCD) and the captured graph (descriptor upload, queue reset,
// persistent kernel) that replays it.
struct BatchSlot {
    BatchDesc* h_desc = nullptr;
    BatchDesc* d_desc = nullptr;
    uint32_t* d_queues = nullptr;
    hipGraph_t graph[kBatchKinds] = {};  // captured on first use of each set of kinds
    hipGraphExec_t exec[kBatchKinds] = {};
    hipEvent_t done = nullptr;
    bool pending = false;
};

// Workgroups of the persistent batch kernels on `device` (index 0: 32 sectors, 1: 128):
// resident blocks per CU times CUs, rounded up to a multiple of the XCD count.
hipError_t batch_grid_size(int device, int grid[2]);
// Allocate a slot's descriptor and queue buffers.
hipError_t init_slot(BatchSlot& s);
// The slot's graph for the set of frame kinds `kinds` (kBatch32 | kBatch128 |
// kBatchHalf), captured on `cap_stream` the first time it is asked for.
hipError_t slot_graph(BatchSlot& s, int kinds, const int grid[2], hipStream_t cap_stream, hipGraphExec_t* exec);
void free_slot(BatchSlot& s);

// The slice-direction table and the sector-boundary tables (32 and 128 sectors) that a
// context uploads, computed on the host.
void fill_tables(int2 lut[kLutSize], double2 half[129], double2 half128[513]);

// Frame constants (FP64 derivation, one rounding to FP32) and the launch shape from
// `tab` (forced, tuned for the frame's class, else the default).
void fill_frame(FrameArgs& A, const FrameTables* tab, const ssvb_image* depth, const ssvb_image* normal,
                const ssvb_image* radiance, const ssvb_camera* cam, const ssvb_params* p, const ssvb_outputs* out);
// Descriptor table of up to kMaxBatch non-empty frames (callers keep it to frames of at
// most kPackTiles tiles): constants, the per-width tile lists and their equal-cost runs.
void build_batch(const FrameTables* tab, BatchDesc* D, const ssvb_frame* frames, int n);

// One frame with the persistent kernel: `queues` is a set of 9 counters that must be
// zero at launch (the kernel leaves them zero when it completes); at most `grid`
// workgroups.
hipError_t launch_plain(const FrameArgs& A, uint32_t* queues, int grid, hipStream_t stream);
int frame_blocks_per_cu();
int slices_blocks_per_cu();
// Multi-bounce light injection (elementwise).
hipError_t launch_inject_bounce(const char* direct, int64_t direct_pitch, int direct_ch, int direct_f16,
                                const char* albedo, int64_t albedo_pitch, int albedo_ch, int albedo_f16,
                                const float* gi, int64_t gi_pitch, char* next, int64_t next_pitch, int next_ch,
                                int next_f16, int W, int H, float gain, hipStream_t stream);
// Slice-major order (A.lp = 1; `partial` holds N_d planes of computed pixels x
// kPartialFloats floats, see partial_off; chunks of `chunk` >= 1 tiles): the per-slice
// gather, then the reduction that writes the outputs; `queues` as for launch_plain.
hipError_t launch_slices(const FrameArgs& A, uint32_t* queues, int grid, float* partial, uint32_t chunk,
                         hipStream_t stream);
// Half resolution: fill the pixels with an odd coordinate from the computed ones.
hipError_t launch_upsample(const FrameArgs& A, hipStream_t stream);
hipError_t launch_debug_lattice(const FrameArgs& A, int32_t* out, hipStream_t stream);
hipError_t launch_debug_endpoints(const FrameArgs& A, float* out, hipStream_t stream);
hipError_t enqueue_batch(const BatchDesc* d_desc, const BatchDesc* h_desc, uint32_t* d_queues, const int grid[2],
                         int kinds, hipStream_t s);
int batch_blocks_per_cu(int sectors);

// Arguments of one denoising pass reading `in` and writing `out`, and the frame constants
// of the half-resolution fill of `out` (inputs already validated by ssvb_denoise).
void fill_denoise(DenoiseArgs& D, const ssvb_image* depth, const ssvb_image* normal, const ssvb_camera* camera,
                  const ssvb_denoise_params* dp, const ssvb_outputs* in, const ssvb_outputs* out);
void fill_upsample(FrameArgs& A, const ssvb_image* depth, const ssvb_camera* camera, const ssvb_outputs* out);

// The argument checks of ssvb_inject_bounce (nothing launched).
ssvb_status validate_bounce(int32_t width, int32_t height, const ssvb_image* direct, const ssvb_image* albedo,
                            const float* gi, int64_t gi_pitch_bytes, float gain, const ssvb_image* next);

// The device and the frame tables of a context.
int ctx_device(const ssvb_ctx* ctx);
const FrameTables* ctx_tables(const ssvb_ctx* ctx);

// Error reporting: the detail goes to the calling thread's last-error string.
ssvb_status fail(ssvb_status s, const char* fmt, ...);
ssvb_status hip_fail(hipError_t e, const char* what);
const std::string& last_error();

// Bytes per element of an ssvb_dtype.
inline int64_t elem_size(int32_t dtype) { return dtype == SSVB_F16 ? 2 : 4; }

}  // namespace ssvb

#endif
