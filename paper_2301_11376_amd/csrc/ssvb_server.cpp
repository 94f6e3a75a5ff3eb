// Request loop of the visibility-bitmask gather: frames are admitted by their HBM
// footprint into a device arena owned by the server (FIFO); buffers in host memory are
// staged through the arena on a copy stream, buffers already in device memory are used
// in place; admitted frames are run in rounds of up to 64 on one or more compute streams
// (one by default; with more, a round can start while another is still on the device).
// A round runs its small frames (at most kPackTiles tiles) in one launch of the batch
// kernel, their tiles packed into one list, and enqueues its larger frames back to back as
// persistent single-frame launches (the fastest kernel for each frame's mode, 128 sectors
// and half resolution included).  Each part of a round (the packed frames, each larger
// frame) ends with an event, so a request is retired, stamped with its completion time and
// its arena block freed as soon as its own part and result copies are done, not at the end
// of its round.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ssvb_host.h"
#include "ssvb_sched.h"

using namespace ssvb;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int kMaxStreams = 8;
constexpr size_t kMaxLive = (size_t)1 << 20;  // tickets not yet released
constexpr uint64_t kAlign = 256;

enum State { QUEUED, RESIDENT, RUNNING, DONE, FAILED };

// Arena layout of one request: the G-buffer as the caller gave it (dense rows) and the
// three FP32 outputs; every part starts on a 256-byte boundary.
struct Layout {
    uint64_t depth, normal, radiance, ao, gi, amb, total;
};

uint64_t up(uint64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

Layout layout_of(const ssvb_frame& F) {
    const uint64_t px = (uint64_t)F.camera.width * (uint64_t)F.camera.height;
    Layout L;
    uint64_t o = 0;
    L.depth = o;
    o += up(px * 4);
    L.normal = o;
    o += up(px * F.normal.channels * elem_size(F.normal.dtype));
    L.radiance = o;
    o += up(px * F.radiance.channels * elem_size(F.radiance.dtype));
    L.ao = o;
    o += up(px * 4);
    L.gi = o;
    o += up(px * 12);
    L.amb = o;
    o += up(px * 12);
    L.total = o;
    return L;
}

struct Request {
    ssvb_frame caller;  // the caller's buffers
    ssvb_frame staged;  // the frame as the kernel reads it: arena copies or the caller's buffers
    Layout lay;
    bool in_place[3] = {};  // depth, normal, radiance already in this device's memory
    bool out_in_place = false;  // all three outputs in this device's memory
    int state = QUEUED;
    ssvb_status err = SSVB_OK;
    Clock::time_point t_submit, t_done;
    // recorded at submission on the caller's stream: the server's copies and kernels for
    // this request wait on it, so they run after everything the caller enqueued before
    hipEvent_t ready = nullptr;
};

// A round on one stream, in parts that finish in stream order: its packed small frames,
// then each larger frame.  Each part's requests are done (results in the caller's
// buffers) when the part's event has fired.
struct Part {
    int ev = 0;  // index into the stream's part events
    std::vector<uint64_t> tickets;
};

struct Round {
    bool busy = false;
    std::vector<uint64_t> tickets;
    std::vector<Part> parts;
    size_t next_part = 0;  // parts before this one have been retired
};

bool terminal(int state) { return state == DONE || state == FAILED; }

int64_t pitch_of(const ssvb_image& im, int W) {
    return im.pitch_bytes ? im.pitch_bytes : (int64_t)W * im.channels * elem_size(im.dtype);
}

}  // namespace

struct ssvb_server {
    int device = 0;
    FrameTables tab;  // the context's device tables and launch shapes, as at creation
    char* arena = nullptr;
    Admission adm;
    int nstreams = 0;
    int grid = 0;  // persistent workgroups of a single-frame launch
    hipStream_t copy_stream = nullptr;
    hipStream_t streams[kMaxStreams] = {};
    hipEvent_t done[kMaxStreams] = {};      // recorded after each round on its stream
    hipEvent_t part_ev[kMaxStreams][kMaxBatch] = {};  // recorded after each part of a round
    uint32_t* counters[kMaxStreams] = {};   // queue counters: one set of 16 per frame of a round
    BatchSlot slot[kMaxStreams];            // the packed small frames of a round, per stream
    int batch_grid[2] = {0, 0};
    Round rounds[kMaxStreams];
    hipEvent_t staged = nullptr;  // recorded on copy_stream after each admission pass

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    hipError_t fatal = hipSuccess;  // first device error; every later request fails with it
    std::string fatal_what;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<hipEvent_t> ev_pool;  // ready events of finished requests, for reuse
    uint64_t next_ticket = 1;
    ssvb_server_counters st{};
};

namespace {

// True if `p` is memory of HIP device `device` (not host memory, pinned or not).
bool on_device(const void* p, int device) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable host memory: not an error for the caller
        return false;
    }
    return at.type == hipMemoryTypeDevice && at.device == device && !at.isManaged;
}

// Point the kernel's view of the request at its arena block, copying in the inputs that
// are not already in device memory (those are read in place).
hipError_t stage(ssvb_server* S, Request& r, uint64_t off) {
    const ssvb_frame& F = r.caller;
    const int W = F.camera.width, H = F.camera.height;
    char* base = S->arena + off;
    r.staged = F;
    const uint64_t at[3] = {r.lay.depth, r.lay.normal, r.lay.radiance};
    ssvb_image* dst[3] = {&r.staged.depth, &r.staged.normal, &r.staged.radiance};
    for (int i = 0; i < 3; ++i) {
        if (r.in_place[i]) continue;
        dst[i]->ptr = base + at[i];
        dst[i]->pitch_bytes = 0;
    }
    if (!r.out_in_place)
        r.staged.out = ssvb_outputs{(float*)(base + r.lay.ao), (float*)(base + r.lay.gi), (float*)(base + r.lay.amb),
                                    nullptr, 0, 0, 0, 0};
    if (!(r.in_place[0] && r.in_place[1] && r.in_place[2])) {
        const hipError_t e = hipStreamWaitEvent(S->copy_stream, r.ready, 0);
        if (e != hipSuccess) return e;
    }
    const ssvb_image* src[3] = {&F.depth, &F.normal, &F.radiance};
    for (int i = 0; i < 3; ++i) {
        if (r.in_place[i]) continue;
        const size_t row = (size_t)W * src[i]->channels * elem_size(src[i]->dtype);
        hipError_t e = hipMemcpy2DAsync((void*)dst[i]->ptr, row, src[i]->ptr, (size_t)pitch_of(*src[i], W), row,
                                        (size_t)H, hipMemcpyDefault, S->copy_stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Copy a request's results from its arena block to the caller's buffers on stream s
// (nothing to do when the kernel wrote the caller's buffers).
hipError_t copy_results(const Request& r, hipStream_t s) {
    if (r.out_in_place) return hipSuccess;
    const ssvb_frame& F = r.caller;
    const int W = F.camera.width, H = F.camera.height;
    struct {
        void* dst;
        int64_t pitch;
        const void* src;
        size_t row;
    } c[3] = {{F.out.ao, F.out.ao_pitch_bytes, r.staged.out.ao, (size_t)W * 4},
              {F.out.gi, F.out.gi_pitch_bytes, r.staged.out.gi, (size_t)W * 12},
              {F.out.ambient, F.out.ambient_pitch_bytes, r.staged.out.ambient, (size_t)W * 12}};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
        e = hipMemcpy2DAsync(c[i].dst, c[i].pitch ? (size_t)c[i].pitch : c[i].row, c[i].src, c[i].row, c[i].row,
                             (size_t)H, hipMemcpyDefault, s);
    return e;
}

// Enqueue a round on stream k: the packed small frames and their result copies, then
// each larger frame and its copies, each part followed by its event.  `parts` receives
// the parts in stream order (tickets[i] is the ticket of rs[i]).
hipError_t launch_round(ssvb_server* S, int k, const std::vector<Request*>& rs, const std::vector<uint64_t>& tickets,
                        std::vector<Part>& parts) {
    hipStream_t s = S->streams[k];
    hipError_t e = hipStreamWaitEvent(s, S->staged, 0);
    // buffers read or written in place (inputs, outputs) are ordered after the caller's work
    for (size_t i = 0; i < rs.size() && e == hipSuccess; ++i) e = hipStreamWaitEvent(s, rs[i]->ready, 0);
    // the stream's previous round has retired: every counter set is back at zero and the
    // slot's descriptor upload is done
    ssvb_frame small[kMaxBatch];
    int n_small = 0, kinds = 0;
    std::vector<size_t> small_i, large_i;
    std::vector<FrameArgs> large;
    large.reserve(rs.size());
    for (size_t i = 0; i < rs.size(); ++i) {
        const ssvb_frame& F = rs[i]->staged;
        FrameArgs A;
        fill_frame(A, &S->tab, &F.depth, &F.normal, &F.radiance, &F.camera, &F.params, &F.out);
        if ((uint32_t)A.tiles_x * (uint32_t)A.tiles_y <= kPackTiles) {
            small[n_small++] = F;
            small_i.push_back(i);
            kinds |= (F.params.sectors == 128 ? kBatch128 : kBatch32) | (F.params.resolution == 2 ? kBatchHalf : 0);
        } else {
            large.push_back(A);
            large_i.push_back(i);
        }
    }
    // larger frames shortest first (tiles x slices x steps): every request but the longest
    // finishes earlier than in arrival order, and the round ends at the same time
    {
        std::vector<size_t> by_cost(large.size());
        for (size_t j = 0; j < by_cost.size(); ++j) by_cost[j] = j;
        auto cost = [&](size_t j) {
            return (double)large[j].tiles_x * large[j].tiles_y * large[j].nd * large[j].ns;
        };
        std::stable_sort(by_cost.begin(), by_cost.end(), [&](size_t a, size_t b) { return cost(a) < cost(b); });
        std::vector<FrameArgs> l2;
        std::vector<size_t> i2;
        for (size_t j : by_cost) {
            l2.push_back(large[j]);
            i2.push_back(large_i[j]);
        }
        large.swap(l2);
        large_i.swap(i2);
    }
    auto finish_part = [&](const std::vector<size_t>& members) {
        for (size_t i : members) {
            if (e != hipSuccess) break;
            e = copy_results(*rs[i], s);
        }
        if (e != hipSuccess) return;
        Part P;
        P.ev = (int)parts.size();
        for (size_t i : members) P.tickets.push_back(tickets[i]);
        e = hipEventRecord(S->part_ev[k][P.ev], s);
        if (e == hipSuccess) parts.push_back(std::move(P));
    };
    if (e == hipSuccess && n_small > 0) {
        // enqueued directly (a graph capture on this thread could collide with a device-wide
        // synchronisation by the caller's threads)
        BatchSlot& B = S->slot[k];
        build_batch(&S->tab, B.h_desc, small, n_small);
        e = enqueue_batch(B.d_desc, B.h_desc, B.d_queues, S->batch_grid, kinds, s);
        finish_part(small_i);
    }
    for (size_t j = 0; j < large.size() && e == hipSuccess; ++j) {
        e = launch_plain(large[j], S->counters[k] + 16 * j, S->grid, s);
        if (e == hipSuccess && large[j].sub == 2) e = launch_upsample(large[j], s);
        if (e == hipSuccess) finish_part({large_i[j]});
    }
    if (e == hipSuccess) e = hipEventRecord(S->done[k], s);
    return e;
}

// A request reached a terminal state: its ready event goes back to the pool (every wait on
// it was enqueued when the request was staged or launched).
void recycle_event(ssvb_server* S, Request& r) {
    if (r.ready) S->ev_pool.push_back(r.ready);
    r.ready = nullptr;
}

void fail_request(ssvb_server* S, uint64_t t, Request& r, Clock::time_point now) {
    recycle_event(S, r);
    r.state = FAILED;
    r.err = SSVB_ERR_DEVICE;
    r.t_done = now;
    S->adm.finish(t);
    S->st.failed++;
}

// The scheduler: retire finished rounds, admit from the queue while memory allows,
// start a round on every idle stream.  HIP calls are made with the lock released; the
// requests they touch are not erased meanwhile (release refuses unfinished tickets).
void run(ssvb_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = false;
        // 1. retire the parts of each round whose events have fired, in stream order; a
        //    round is over (its stream idle) once its last event has fired.  Only this
        //    thread touches the rounds, so their events are queried with the lock released.
        int running = 0;
        for (int k = 0; k < S->nstreams; ++k) {
            Round& R = S->rounds[k];
            if (!R.busy) continue;
            hipError_t qs[kMaxBatch];
            int nq = 0;
            hipError_t qd = hipErrorNotReady;
            lk.unlock();
            size_t p = R.next_part;
            for (; p < R.parts.size(); ++p) {
                qs[nq] = hipEventQuery(S->part_ev[k][R.parts[p].ev]);
                if (qs[nq++] != hipSuccess) break;
            }
            if (p == R.parts.size()) qd = hipEventQuery(S->done[k]);
            bool bad = qd != hipSuccess && qd != hipErrorNotReady;
            for (int i = 0; i < nq; ++i) bad = bad || (qs[i] != hipSuccess && qs[i] != hipErrorNotReady);
            // before the round's requests are failed (and their buffers possibly freed by
            // the caller), let whatever of it is still in flight drain
            if (bad) (void)hipStreamSynchronize(S->streams[k]);
            lk.lock();
            const Clock::time_point now = Clock::now();
            hipError_t err = hipSuccess;
            for (int i = 0; i < nq && qs[i] != hipErrorNotReady; ++i) {
                if (qs[i] != hipSuccess) {
                    err = qs[i];
                    break;
                }
                for (uint64_t t : R.parts[R.next_part].tickets) {
                    Request& r = S->reqs[t];
                    recycle_event(S, r);
                    r.state = DONE;
                    r.t_done = now;
                    S->adm.finish(t);
                    S->st.completed++;
                }
                ++R.next_part;
                progress = true;
            }
            if (err == hipSuccess && qd != hipSuccess && qd != hipErrorNotReady) err = qd;
            if (err != hipSuccess) {
                for (; R.next_part < R.parts.size(); ++R.next_part)
                    for (uint64_t t : R.parts[R.next_part].tickets) fail_request(S, t, S->reqs[t], now);
                if (S->fatal == hipSuccess) {
                    S->fatal = err;
                    S->fatal_what = "round";
                }
            }
            if (err != hipSuccess || (R.next_part == R.parts.size() && qd == hipSuccess)) {
                R.busy = false;
                R.tickets.clear();
                R.parts.clear();
                R.next_part = 0;
                progress = true;
            } else {
                ++running;
            }
        }
        if (progress) S->cv_done.notify_all();
        if (S->stop) {
            if (running == 0) break;
            S->cv_work.wait_for(lk, std::chrono::microseconds(50));
            continue;
        }
        // 2. admit in arrival order while the head fits; 3. one round per idle stream
        std::vector<std::pair<uint64_t, uint64_t>> admitted;
        std::vector<std::pair<int, std::vector<uint64_t>>> starts;
        if (S->fatal == hipSuccess) {
            S->adm.admit(admitted);
            for (auto& a : admitted) {
                S->reqs[a.first].state = RESIDENT;
                if (running > 0) S->st.admitted_while_running++;
            }
            for (int k = 0; k < S->nstreams && S->adm.ready() > 0; ++k) {
                if (S->rounds[k].busy) continue;
                std::vector<uint64_t> tk;
                S->adm.take_round(tk);
                for (uint64_t t : tk) S->reqs[t].state = RUNNING;
                S->rounds[k].busy = true;
                S->rounds[k].tickets = tk;
                S->st.rounds++;
                S->st.frames_in_rounds += tk.size();
                if ((int32_t)tk.size() > S->st.max_round_frames) S->st.max_round_frames = (int32_t)tk.size();
                starts.push_back({k, std::move(tk)});
                ++running;
            }
            if (running > S->st.max_running_rounds) S->st.max_running_rounds = running;
        }
        if (admitted.empty() && starts.empty()) {
            if (running > 0) S->cv_work.wait_for(lk, std::chrono::microseconds(50));
            else if (!progress) S->cv_work.wait(lk);
            continue;
        }
        std::vector<Request*> adm_req;
        for (auto& a : admitted) adm_req.push_back(&S->reqs[a.first]);
        std::vector<std::vector<Request*>> round_req;
        for (auto& s : starts) {
            round_req.emplace_back();
            for (uint64_t t : s.second) round_req.back().push_back(&S->reqs[t]);
        }
        lk.unlock();
        hipError_t e = hipSuccess;
        for (size_t i = 0; i < admitted.size() && e == hipSuccess; ++i) e = stage(S, *adm_req[i], admitted[i].second);
        if (!admitted.empty() && e == hipSuccess) e = hipEventRecord(S->staged, S->copy_stream);
        const char* what = "staging";
        std::vector<std::vector<Part>> parts(starts.size());
        for (size_t i = 0; i < starts.size() && e == hipSuccess; ++i) {
            e = launch_round(S, starts[i].first, round_req[i], starts[i].second, parts[i]);
            what = "round launch";
        }
        if (e != hipSuccess) {
            // the requests below are about to be failed: first let the copies and rounds
            // already enqueued for them finish, so nothing on the device still reads or
            // writes their buffers once the caller sees them failed
            (void)hipStreamSynchronize(S->copy_stream);
            for (auto& s : starts) (void)hipStreamSynchronize(S->streams[s.first]);
        }
        lk.lock();
        for (size_t i = 0; i < starts.size() && e == hipSuccess; ++i) {
            Round& R = S->rounds[starts[i].first];
            R.parts = std::move(parts[i]);
            R.next_part = 0;
        }
        if (e != hipSuccess) {
            // a device error leaves the server unusable: fail everything not yet retired
            if (S->fatal == hipSuccess) {
                S->fatal = e;
                S->fatal_what = what;
            }
            const Clock::time_point t_fail = Clock::now();
            for (auto& s : starts) {
                for (uint64_t t : s.second) fail_request(S, t, S->reqs[t], t_fail);
                Round& R = S->rounds[s.first];
                R.busy = false;
                R.tickets.clear();
                R.parts.clear();
                R.next_part = 0;
            }
            for (uint64_t t : S->adm.cancel_ready()) fail_request(S, t, S->reqs[t], t_fail);
            for (uint64_t t : S->adm.cancel_queued()) {
                Request& r = S->reqs[t];
                recycle_event(S, r);
                r.state = FAILED;
                r.err = SSVB_ERR_DEVICE;
                r.t_done = t_fail;
                S->st.failed++;
            }
            S->cv_done.notify_all();
        }
    }
}

ssvb_status fatal_status(const ssvb_server* S) {
    return fail(SSVB_ERR_DEVICE, "server stopped after a device error (%s): %s", S->fatal_what.c_str(),
                hipGetErrorString(S->fatal));
}

void destroy_resources(ssvb_server* S) {
    for (auto& kv : S->reqs)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    for (hipEvent_t ev : S->ev_pool) (void)hipEventDestroy(ev);
    S->ev_pool.clear();
    for (int k = 0; k < kMaxStreams; ++k) {
        for (int i = 0; i < kMaxBatch; ++i)
            if (S->part_ev[k][i]) (void)hipEventDestroy(S->part_ev[k][i]);
        free_slot(S->slot[k]);
        if (S->done[k]) (void)hipEventDestroy(S->done[k]);
        if (S->counters[k]) (void)hipFree(S->counters[k]);
        if (S->streams[k]) (void)hipStreamDestroy(S->streams[k]);
    }
    if (S->staged) (void)hipEventDestroy(S->staged);
    if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
    if (S->arena) (void)hipFree(S->arena);
}

}  // namespace

extern "C" {

ssvb_status ssvb_server_create(ssvb_ctx* ctx, uint64_t hbm_budget_bytes, int32_t streams, ssvb_server** out) {
    if (!out) return fail(SSVB_ERR_INVALID_ARG, "NULL output handle");
    *out = nullptr;
    if (!ctx) return fail(SSVB_ERR_INVALID_ARG, "NULL context");
    if (streams == 0) streams = 1;
    if (streams < 1 || streams > kMaxStreams)
        return fail(SSVB_ERR_INVALID_ARG, "streams %d outside [1, %d]", streams, kMaxStreams);
    if (hbm_budget_bytes < kAlign) return fail(SSVB_ERR_INVALID_ARG, "HBM budget of %llu bytes is too small",
                                               (unsigned long long)hbm_budget_bytes);
    ssvb_server* S = new (std::nothrow) ssvb_server();
    if (!S) return fail(SSVB_ERR_OUT_OF_MEMORY, "host allocation");
    S->device = ctx_device(ctx);
    S->tab = *ctx_tables(ctx);
    S->nstreams = streams;
    S->adm = Admission(hbm_budget_bytes, kMaxBatch, kAlign);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    hipError_t e = hipMalloc((void**)&S->arena, S->adm.arena().size());
    const bool oom = e == hipErrorOutOfMemory;
    if (e == hipSuccess) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, S->device);
        S->grid = prop.multiProcessorCount * frame_blocks_per_cu();
    }
    if (e == hipSuccess) e = batch_grid_size(S->device, S->batch_grid);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->staged, hipEventDisableTiming);
    for (int k = 0; k < streams && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&S->streams[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->done[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc((void**)&S->counters[k], kMaxBatch * 16 * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemset(S->counters[k], 0, kMaxBatch * 16 * sizeof(uint32_t));
        if (e == hipSuccess) e = init_slot(S->slot[k]);
        for (int i = 0; i < kMaxBatch && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&S->part_ev[k][i], hipEventDisableTiming);
    }
    // a round waits on `staged` even before anything was staged: record it once
    if (e == hipSuccess) e = hipEventRecord(S->staged, S->copy_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->copy_stream);
    if (e != hipSuccess) {
        destroy_resources(S);
        (void)hipSetDevice(prev);
        delete S;
        return oom ? fail(SSVB_ERR_OUT_OF_MEMORY, "arena of %llu bytes", (unsigned long long)hbm_budget_bytes)
                   : hip_fail(e, "server set-up");
    }
    (void)hipSetDevice(prev);
    S->st.arena_bytes = S->adm.arena().size();
    try {
        S->worker = std::thread(run, S);
    } catch (...) {
        destroy_resources(S);
        delete S;
        return fail(SSVB_ERR_OUT_OF_MEMORY, "scheduler thread");
    }
    *out = S;
    return SSVB_OK;
}

ssvb_status ssvb_server_submit(ssvb_server* S, const ssvb_frame* frame, void* hip_stream, uint64_t* ticket) {
    if (!S || !frame || !ticket) return fail(SSVB_ERR_INVALID_ARG, "NULL argument");
    const ssvb_frame& F = *frame;
    ssvb_status s = ssvb_validate(&F.depth, &F.normal, &F.radiance, &F.camera, &F.params, &F.out);
    if (s) return s;
    if (F.out.masks) return fail(SSVB_ERR_INVALID_ARG, "served requests do not return slice masks");
    Request r;
    r.caller = F;
    r.lay = layout_of(F);
    if ((int64_t)F.camera.width * F.camera.height > 0) {
        r.in_place[0] = on_device(F.depth.ptr, S->device);
        r.in_place[1] = on_device(F.normal.ptr, S->device);
        r.in_place[2] = on_device(F.radiance.ptr, S->device);
        r.out_in_place = on_device(F.out.ao, S->device) && on_device(F.out.gi, S->device) &&
                         on_device(F.out.ambient, S->device);
    }
    if (!S->adm.fits_at_all(r.lay.total))
        return fail(SSVB_ERR_OUT_OF_MEMORY, "request footprint %llu bytes exceeds the %llu-byte arena",
                    (unsigned long long)r.lay.total, (unsigned long long)S->adm.arena().size());
    const bool empty = (int64_t)F.camera.width * F.camera.height == 0;
    if (!empty) {
        // order the request after the caller's work on `hip_stream`
        {
            std::lock_guard<std::mutex> g(S->mu);
            if (!S->ev_pool.empty()) {
                r.ready = S->ev_pool.back();
                S->ev_pool.pop_back();
            }
        }
        int prev = 0;
        (void)hipGetDevice(&prev);
        if (prev != S->device) (void)hipSetDevice(S->device);
        hipError_t e = r.ready ? hipSuccess : hipEventCreateWithFlags(&r.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r.ready, (hipStream_t)hip_stream);
        if (prev != S->device) (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            if (r.ready) {
                std::lock_guard<std::mutex> g(S->mu);
                S->ev_pool.push_back(r.ready);
            }
            return hip_fail(e, "recording the request's ready event");
        }
    }
    {
        std::lock_guard<std::mutex> g(S->mu);
        auto refuse = [&](ssvb_status st) {
            recycle_event(S, r);
            return st;
        };
        if (S->fatal != hipSuccess) return refuse(fatal_status(S));
        if (S->stop) return refuse(fail(SSVB_ERR_BUSY, "server is shutting down"));
        if (S->reqs.size() >= kMaxLive)
            return refuse(fail(SSVB_ERR_BUSY, "%zu requests not yet released", S->reqs.size()));
        const uint64_t t = S->next_ticket++;
        r.t_submit = Clock::now();
        if (empty) {
            r.state = DONE;
            r.t_done = r.t_submit;
            S->st.completed++;
        } else {
            S->adm.submit(t, r.lay.total);
        }
        S->reqs.emplace(t, r);
        S->st.submitted++;
        *ticket = t;
    }
    S->cv_work.notify_one();
    return SSVB_OK;
}

ssvb_status ssvb_server_poll(ssvb_server* S, uint64_t ticket, int32_t* done, double* latency_ms) {
    if (!S || !done) return fail(SSVB_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(SSVB_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    const Request& r = it->second;
    *done = terminal(r.state) ? 1 : 0;
    if (latency_ms) *latency_ms = *done ? std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count() : 0.0;
    if (r.state == FAILED) return fail(r.err, "request %llu failed on the device", (unsigned long long)ticket);
    return SSVB_OK;
}

ssvb_status ssvb_server_wait(ssvb_server* S, uint64_t ticket, double timeout_ms, double* latency_ms) {
    if (!S) return fail(SSVB_ERR_INVALID_ARG, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(SSVB_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = &it->second;
    auto finished = [&] { return terminal(r->state); };
    if (timeout_ms < 0) {
        S->cv_done.wait(lk, finished);
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), finished)) {
        return fail(SSVB_ERR_TIMEOUT, "request %llu not finished after %.3f ms", (unsigned long long)ticket, timeout_ms);
    }
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    if (r->state == FAILED) return fail(r->err, "request %llu failed on the device", (unsigned long long)ticket);
    return SSVB_OK;
}

ssvb_status ssvb_server_release(ssvb_server* S, uint64_t ticket) {
    if (!S) return fail(SSVB_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(SSVB_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (!terminal(it->second.state)) return fail(SSVB_ERR_BUSY, "request %llu has not finished", (unsigned long long)ticket);
    S->reqs.erase(it);
    return SSVB_OK;
}

ssvb_status ssvb_server_stats(ssvb_server* S, ssvb_server_counters* out) {
    if (!S || !out) return fail(SSVB_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    *out = S->st;
    out->arena_in_use = S->adm.arena().in_use();
    out->arena_peak = S->adm.arena().peak();
    out->queued = (int32_t)S->adm.queued();
    out->resident = (int32_t)S->adm.resident();
    int running = 0;
    for (int k = 0; k < S->nstreams; ++k) running += S->rounds[k].busy;
    out->running_rounds = running;
    return SSVB_OK;
}

ssvb_status ssvb_server_destroy(ssvb_server* S) {
    if (!S) return SSVB_OK;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
        // requests not yet in a round are dropped; rounds on the device are waited for
        for (uint64_t t : S->adm.cancel_ready()) S->reqs[t].state = FAILED;
        for (uint64_t t : S->adm.cancel_queued()) {
            recycle_event(S, S->reqs[t]);
            S->reqs[t].state = FAILED;
        }
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    hipError_t e = hipStreamSynchronize(S->copy_stream);  // staging of dropped requests
    for (int k = 0; k < S->nstreams; ++k) {
        const hipError_t e2 = hipStreamSynchronize(S->streams[k]);
        if (e == hipSuccess) e = e2;
    }
    destroy_resources(S);
    (void)hipSetDevice(prev);
    delete S;
    if (e != hipSuccess) return hip_fail(e, "server shutdown");
    return SSVB_OK;
}

}  // extern "C"
