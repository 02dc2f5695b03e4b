// server.hip -- continuous-batching request loop (host scheduler + batched ray-march launches).
//
// The paper renders asynchronously so that the display never waits for the
// volume renderer (Section 2.2).  Here a scheduler thread owned by the context
// keeps the volumes resident and serves many render requests at once:
//
//  * submit (any thread) validates a request exactly like raypc_render and
//    captures its brush, transfer function and kernel arguments; it then waits
//    in a FIFO queue;
//  * admission takes requests in submission order while a request slot is free
//    and the memory budget (image bytes + skip flags) allows; admitting uploads
//    the request's kernel arguments and table to its slot and computes its
//    sub-brick skip flags on the upload stream;
//  * every step is one batched launch (one per storage type present) over
//    tile ranges of the admitted requests, oldest first, up to tiles_per_step
//    tiles; the ranges travel in the kernel arguments, so a step copies
//    nothing.  Requests admitted meanwhile join the next step, so work of many
//    requests overlaps on the device;
//  * steps alternate between two streams that wait for the upload stream only
//    when something was uploaded since they last did: a step's blocks start
//    while the previous step's last blocks still run, instead of the device
//    draining at every step boundary;
//  * steps are recorded with events and retired in launch order; a request is
//    done when the steps up to the one holding its last tile have completed,
//    and its slot and budget are released.
//
// Device memory is allocated once at server start (per-slot arguments, tables
// and skip flags); nothing is allocated or freed per request.  Waiting uses
// event queries, short condition-variable waits and hipEventSynchronize when
// the device queue is full.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "context.h"
#include "internal.h"
#include "server.h"

namespace raypc {
namespace {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kMaxSlots = 256;
constexpr size_t kMaxSkipWords = 128u * 128u * 128u;  // flag words of a level with 128^3 bricks
constexpr int kDefaultTilesPerStep = 32768;

struct Request {
    uint64_t ticket = 0;
    int state = RAYPC_REQ_QUEUED;  // or -RAYPC_ERR_*
    double deadline = 0.0;         // absolute, ms; 0: none
    double t[4] = {0, 0, 0, 0};
    RenderArgs args{};             // complete except the per-slot skip / table pointers
    SkipArgs skip_args{};          // complete except the output pointers
    float tf_rgba[RAYPC_TF_ENTRIES * 4];
    int storage = 0;  // kernel kind
    int nb_class = 0;  // field-count class of its launches (batch_nb_class)
    bool wide = false;  // 64-bit record offsets (batch_wide)
    int n_tiles = 0, next_tile = 0;
    uint64_t bytes = 0;
    int slot = -1;
    Volume* vol = nullptr;
};

struct Step {
    hipEvent_t done = nullptr;
    std::vector<Request*> finishing;
};

}  // namespace

struct Server {
    raypc_ctx* ctx = nullptr;
    raypc_server_cfg cfg{};
    std::thread thread;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stopping = false;
    uint64_t next_ticket = 1;
    std::deque<Request*> queue;
    std::vector<Request*> active;  // admitted, in admission order
    std::unordered_map<uint64_t, Request*> all;
    std::vector<int> free_slots;
    std::deque<Step> steps;
    std::vector<hipEvent_t> events;
    raypc_server_stats stats{};
    hipStream_t upload = nullptr;          // argument / table uploads and skip flags
    hipStream_t step_stream[2] = {nullptr, nullptr};
    hipEvent_t uploaded = nullptr;         // recorded on `upload` after each admission round
    uint64_t upload_seq = 0;               // admission rounds recorded so far
    uint64_t waited_seq[2] = {0, 0};       // last round each step stream waited for
    uint64_t n_launched = 0;
    RenderArgs* d_args = nullptr;
    RenderArgs* h_args = nullptr;
    float4* d_tf = nullptr;
    float4* h_tf = nullptr;
    uint16_t* d_skip = nullptr;
    int fatal = 0;  // set when a device call failed: every later request fails with it
};

namespace {

void release_volume_ref(Server* S, Request* r) {
    std::lock_guard<std::mutex> lk(S->ctx->mu);
    if (r->vol) r->vol->refs -= 1;
    r->vol = nullptr;
}

// Finish a request that never reached the device (timeout, cancel, failure before admission).
void end_unadmitted(Server* S, Request* r, int code) {
    r->state = -code;
    r->t[3] = now_ms();
    release_volume_ref(S, r);
    if (code == RAYPC_ERR_TIMEOUT) S->stats.timed_out++;
    else if (code == RAYPC_ERR_CANCELLED) S->stats.cancelled++;
    else S->stats.failed++;
    S->cv_done.notify_all();
}

void finish_admitted(Server* S, Request* r, int code, double t) {
    r->state = code == RAYPC_OK ? RAYPC_REQ_DONE : -code;
    r->t[3] = t;
    S->free_slots.push_back(r->slot);
    S->stats.bytes_in_use -= r->bytes;
    S->active.erase(std::find(S->active.begin(), S->active.end(), r));
    release_volume_ref(S, r);
    if (code == RAYPC_OK) S->stats.completed++;
    else S->stats.failed++;
}

void fail_everything_active(Server* S, int code) {
    const double t = now_ms();
    for (auto& st : S->steps)
        if (st.done) S->events.push_back(st.done);
    S->steps.clear();
    while (!S->active.empty()) finish_admitted(S, S->active.front(), code, t);
    S->fatal = code;
    S->cv_done.notify_all();
}

// Completed steps -> completed requests.
void retire(Server* S) {
    while (!S->steps.empty()) {
        const hipError_t e = hipEventQuery(S->steps.front().done);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail_everything_active(S, RAYPC_ERR_DEVICE);
            return;
        }
        Step st = S->steps.front();
        S->steps.pop_front();
        const double t = now_ms();
        for (Request* r : st.finishing) finish_admitted(S, r, RAYPC_OK, t);
        S->events.push_back(st.done);
        S->cv_done.notify_all();
    }
}

void admit(Server* S) {
    bool any = false;
    while (!S->queue.empty()) {
        Request* r = S->queue.front();
        if (r->state != RAYPC_REQ_QUEUED) {  // cancelled while queued
            S->queue.pop_front();
            continue;
        }
        if (S->fatal) {
            S->queue.pop_front();
            end_unadmitted(S, r, S->fatal);
            continue;
        }
        if (r->deadline > 0.0 && now_ms() > r->deadline) {
            S->queue.pop_front();
            end_unadmitted(S, r, RAYPC_ERR_TIMEOUT);
            continue;
        }
        if (S->free_slots.empty()) break;
        if (S->cfg.mem_budget_bytes && S->stats.bytes_in_use + r->bytes > S->cfg.mem_budget_bytes) break;
        S->queue.pop_front();
        const int slot = S->free_slots.back();
        S->free_slots.pop_back();
        RenderArgs a = r->args;
        a.skip = S->d_skip + static_cast<size_t>(slot) * kMaxSkipWords;
        a.tf = S->d_tf + static_cast<size_t>(slot) * RAYPC_TF_ENTRIES;
        S->h_args[slot] = a;
        std::memcpy(S->h_tf + static_cast<size_t>(slot) * RAYPC_TF_ENTRIES, r->tf_rgba, sizeof(r->tf_rgba));
        SkipArgs sk = r->skip_args;
        sk.out_sub = const_cast<uint16_t*>(a.skip);
        hipError_t e = hipMemcpyAsync(S->d_args + slot, S->h_args + slot, sizeof(RenderArgs), hipMemcpyHostToDevice,
                                      S->upload);
        if (e == hipSuccess)
            e = hipMemcpyAsync(const_cast<float4*>(a.tf), S->h_tf + static_cast<size_t>(slot) * RAYPC_TF_ENTRIES,
                               sizeof(r->tf_rgba), hipMemcpyHostToDevice, S->upload);
        if (e == hipSuccess) e = launch_skip(sk, S->upload);
        any = true;
        r->slot = slot;
        r->state = RAYPC_REQ_RUNNING;
        r->t[1] = now_ms();
        S->stats.bytes_in_use += r->bytes;
        S->stats.peak_bytes_in_use = std::max(S->stats.peak_bytes_in_use, S->stats.bytes_in_use);
        S->active.push_back(r);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail_everything_active(S, RAYPC_ERR_DEVICE);
            return;
        }
    }
    if (any) {
        if (hipEventRecord(S->uploaded, S->upload) != hipSuccess) {
            (void)hipGetLastError();
            fail_everything_active(S, RAYPC_ERR_DEVICE);
            return;
        }
        S->upload_seq++;
    }
}

bool has_pending_tiles(const Server* S) {
    for (const Request* r : S->active)
        if (r->next_tile < r->n_tiles) return true;
    return false;
}

// One batched step: tile ranges of the admitted requests, oldest first, one launch per kernel kind,
// field-count class and record offset width present (more if one has more ranges than a launch
// carries).
void launch_step(Server* S) {
    struct Take {
        Request* r;
        int start, count;
    };
    std::vector<Take> takes;
    // the budget counts 8x8-pixel units; the renderer's tiles are 4x4 pixels
    int budget = S->cfg.tiles_per_step * (8 / kBlockPix) * (8 / kBlockPix);
    for (Request* r : S->active) {
        if (budget == 0) break;
        const int left = r->n_tiles - r->next_tile;
        if (left <= 0) continue;
        const int c = std::min(left, budget);
        takes.push_back({r, r->next_tile, c});
        budget -= c;
    }
    const int which = static_cast<int>(S->n_launched & 1u);
    hipStream_t s = S->step_stream[which];
    hipError_t e = hipSuccess;
    if (S->waited_seq[which] != S->upload_seq) {
        e = hipStreamWaitEvent(s, S->uploaded, 0);
        S->waited_seq[which] = S->upload_seq;
    }
    int k = 0;
    for (int kind = 0; kind < kKinds && e == hipSuccess; ++kind) {
        for (int cls = 0; cls < 2 * (kMaxFields + 2) && e == hipSuccess; ++cls) {
            const int nb = cls % (kMaxFields + 2) - 1;
            const bool wide = cls >= kMaxFields + 2;
            BatchRanges R;
            R.n = 0;
            int items = 0;
            for (const Take& t : takes) {
                if (t.r->storage != kind || t.r->nb_class != nb || t.r->wide != wide) continue;
                if (R.n == kMaxRanges) {
                    e = launch_render_batch(S->d_args, R, kind, nb, wide, s);
                    if (e != hipSuccess) break;
                    R.n = 0;
                    items = 0;
                }
                items += t.count;
                R.end[R.n] = items;
                R.first[R.n] = t.start;
                R.slot[R.n] = t.r->slot;
                R.n++;
                k += t.count;
            }
            if (e == hipSuccess && R.n) e = launch_render_batch(S->d_args, R, kind, nb, wide, s);
        }
    }
    Step step;
    if (S->events.empty()) {
        hipEvent_t ev;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) S->events.push_back(ev);
    }
    if (e == hipSuccess) {
        step.done = S->events.back();
        S->events.pop_back();
        e = hipEventRecord(step.done, s);
    }
    const double t = now_ms();
    for (const Take& tk : takes) {
        if (tk.start == 0) tk.r->t[2] = t;
        tk.r->next_tile += tk.count;
        if (tk.r->next_tile == tk.r->n_tiles) step.finishing.push_back(tk.r);
    }
    S->steps.push_back(step);
    S->n_launched++;
    S->stats.steps++;
    S->stats.tiles += static_cast<uint64_t>(k);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail_everything_active(S, RAYPC_ERR_DEVICE);
    }
}

void run(Server* S) {
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        retire(S);
        admit(S);
        const bool pending = has_pending_tiles(S);
        if (pending && static_cast<int>(S->steps.size()) < S->cfg.steps_in_flight) {
            launch_step(S);
            continue;
        }
        if (S->stopping && S->queue.empty() && S->active.empty() && S->steps.empty()) break;
        if (pending || (!S->steps.empty() && S->queue.empty())) {
            // device queue full, or only completions to wait for: block on the oldest step
            hipEvent_t ev = S->steps.front().done;
            lk.unlock();
            (void)hipEventSynchronize(ev);
            lk.lock();
        } else if (!S->steps.empty()) {
            // queued requests wait for memory or slots that the running steps will free
            S->cv_work.wait_for(lk, std::chrono::microseconds(50));
        } else if (S->queue.empty()) {
            S->cv_work.wait(lk, [S] { return S->stopping || !S->queue.empty(); });
        } else {
            // requests queued but none admissible and nothing running: only deadlines can move them
            S->cv_work.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

void free_resources(Server* S) {
    for (hipEvent_t e : S->events) (void)hipEventDestroy(e);
    for (auto& st : S->steps)
        if (st.done) (void)hipEventDestroy(st.done);
    if (S->uploaded) (void)hipEventDestroy(S->uploaded);
    if (S->upload) (void)hipStreamDestroy(S->upload);
    for (hipStream_t st : S->step_stream)
        if (st) (void)hipStreamDestroy(st);
    (void)hipFree(S->d_args);
    (void)hipFree(S->d_tf);
    (void)hipFree(S->d_skip);
    (void)hipHostFree(S->h_args);
    (void)hipHostFree(S->h_tf);
    for (auto& kv : S->all) delete kv.second;
    delete S;
}

Server* get_server(raypc_ctx* ctx) { return ctx ? ctx->server : nullptr; }

}  // namespace

void server_shutdown(raypc_ctx* ctx) {
    Server* S = ctx->server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    if (S->thread.joinable()) S->thread.join();
    ctx->server = nullptr;
    free_resources(S);
}

}  // namespace raypc

using namespace raypc;

extern "C" {

int raypc_server_start(raypc_ctx* ctx, const raypc_server_cfg* cfg) {
    if (!ctx || !cfg) return set_error(RAYPC_ERR_INVALID, "NULL argument");
    if (ctx->server) return set_error(RAYPC_ERR_STATE, "a server is already running on this context");
    raypc_server_cfg c = *cfg;
    if (c.max_inflight < 1 || c.max_inflight > kMaxSlots)
        return set_error(RAYPC_ERR_INVALID, "max_inflight %d outside [1, %d]", c.max_inflight, kMaxSlots);
    if (c.tiles_per_step == 0) c.tiles_per_step = kDefaultTilesPerStep;
    if (c.tiles_per_step < 1 || c.tiles_per_step > (1 << 20))
        return set_error(RAYPC_ERR_INVALID, "tiles_per_step %d outside [1, 2^20]", c.tiles_per_step);
    if (c.steps_in_flight == 0) c.steps_in_flight = 2;
    if (c.steps_in_flight < 1 || c.steps_in_flight > 4)
        return set_error(RAYPC_ERR_INVALID, "steps_in_flight %d outside [1, 4]", c.steps_in_flight);
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    Server* S = new Server();
    S->ctx = ctx;
    S->cfg = c;
    const size_t slots = static_cast<size_t>(c.max_inflight);
    hipError_t e = hipStreamCreateWithFlags(&S->upload, hipStreamNonBlocking);
    for (hipStream_t& st : S->step_stream)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->uploaded, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->d_args), slots * sizeof(RenderArgs));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->d_tf), slots * RAYPC_TF_ENTRIES * sizeof(float4));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->d_skip), slots * kMaxSkipWords * sizeof(uint16_t));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S->h_args), slots * sizeof(RenderArgs), 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S->h_tf), slots * RAYPC_TF_ENTRIES * sizeof(float4), 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_resources(S);
        if (prev >= 0) (void)hipSetDevice(prev);
        return set_error(e == hipErrorOutOfMemory ? RAYPC_ERR_NOMEM : RAYPC_ERR_DEVICE, "server start: %s",
                         hipGetErrorString(e));
    }
    for (int i = c.max_inflight - 1; i >= 0; --i) S->free_slots.push_back(i);
    ctx->server = S;
    S->thread = std::thread(run, S);
    if (prev >= 0) (void)hipSetDevice(prev);
    return RAYPC_OK;
}

int raypc_server_stop(raypc_ctx* ctx) {
    if (!ctx) return set_error(RAYPC_ERR_INVALID, "ctx is NULL");
    if (!ctx->server) return set_error(RAYPC_ERR_STATE, "no server is running");
    server_shutdown(ctx);
    return RAYPC_OK;
}

int raypc_submit(raypc_ctx* ctx, const raypc_request* req, uint64_t* ticket) {
    if (!ctx || !req || !ticket) return set_error(RAYPC_ERR_INVALID, "NULL argument");
    Server* S = get_server(ctx);
    if (!S) return set_error(RAYPC_ERR_STATE, "no server is running");
    Request* r = new Request();
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        int level = 0;
        Volume* v = nullptr;
        CoordBrush coord;
        for (int ax = 0; ax < 4; ++ax) {
            coord.active[ax] = req->coord_active[ax];
            coord.lo[ax] = req->coord_lo[ax];
            coord.hi[ax] = req->coord_hi[ax];
        }
        const int rc = prepare_render(ctx, req->volume_id, &req->camera, req->width, req->height, req->lod, req->step,
                                      req->active, req->lo, req->hi, coord, req->tf_slot, req->out, false, nullptr,
                                      r->args, r->storage, level, &v);
        if (rc) {
            delete r;
            return rc;
        }
        r->nb_class = batch_nb_class(r->args);
        r->wide = batch_wide(r->args, r->storage);
        build_skip_args(ctx, v, level, req->active, req->lo, req->hi, coord, req->tf_slot, r->skip_args);
        std::memcpy(r->tf_rgba, ctx->tf[req->tf_slot].rgba, sizeof(r->tf_rgba));
        r->n_tiles = r->args.n_blocks;
        r->bytes = static_cast<uint64_t>(req->width) * req->height * 16u +
                   static_cast<uint64_t>(r->skip_args.n_bricks) * sizeof(uint16_t);
        if (S->cfg.mem_budget_bytes && r->bytes > S->cfg.mem_budget_bytes) {
            delete r;
            return set_error(RAYPC_ERR_NOMEM, "request needs %llu bytes, the server budget is %llu",
                             static_cast<unsigned long long>(r->bytes),
                             static_cast<unsigned long long>(S->cfg.mem_budget_bytes));
        }
        v->refs += 1;
        r->vol = v;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping) {
            release_volume_ref(S, r);
            delete r;
            return set_error(RAYPC_ERR_STATE, "the server is stopping");
        }
        r->ticket = S->next_ticket++;
        r->t[0] = now_ms();
        if (req->deadline_ms > 0.0) r->deadline = r->t[0] + req->deadline_ms;
        S->all[r->ticket] = r;
        S->queue.push_back(r);
        S->stats.submitted++;
        *ticket = r->ticket;
    }
    S->cv_work.notify_one();
    return RAYPC_OK;
}

int raypc_poll(raypc_ctx* ctx, uint64_t ticket, int* state) {
    Server* S = get_server(ctx);
    if (!S || !state) return set_error(S ? RAYPC_ERR_INVALID : RAYPC_ERR_STATE, "no server or NULL state");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return set_error(RAYPC_ERR_INVALID, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
    *state = it->second->state;
    return RAYPC_OK;
}

int raypc_wait(raypc_ctx* ctx, uint64_t ticket, int timeout_ms) {
    Server* S = get_server(ctx);
    if (!S) return set_error(RAYPC_ERR_STATE, "no server is running");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return set_error(RAYPC_ERR_INVALID, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
    Request* r = it->second;
    auto finished = [r] { return r->state == RAYPC_REQ_DONE || r->state < 0; };
    if (timeout_ms < 0) {
        S->cv_done.wait(lk, finished);
    } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished)) {
        return set_error(RAYPC_ERR_TIMEOUT, "request %llu not done after %d ms", static_cast<unsigned long long>(ticket),
                         timeout_ms);
    }
    if (r->state < 0) return set_error(-r->state, "request %llu ended with error %d", static_cast<unsigned long long>(ticket),
                                       -r->state);
    return RAYPC_OK;
}

int raypc_cancel(raypc_ctx* ctx, uint64_t ticket) {
    Server* S = get_server(ctx);
    if (!S) return set_error(RAYPC_ERR_STATE, "no server is running");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return set_error(RAYPC_ERR_INVALID, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
    Request* r = it->second;
    if (r->state != RAYPC_REQ_QUEUED) return set_error(RAYPC_ERR_BUSY, "request already admitted or finished");
    end_unadmitted(S, r, RAYPC_ERR_CANCELLED);  // the queue entry is dropped by the scheduler
    return RAYPC_OK;
}

int raypc_request_times(raypc_ctx* ctx, uint64_t ticket, double times_ms[4]) {
    Server* S = get_server(ctx);
    if (!S || !times_ms) return set_error(S ? RAYPC_ERR_INVALID : RAYPC_ERR_STATE, "no server or NULL output");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return set_error(RAYPC_ERR_INVALID, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
    for (int k = 0; k < 4; ++k) times_ms[k] = it->second->t[k];
    return RAYPC_OK;
}

int raypc_release(raypc_ctx* ctx, uint64_t ticket) {
    Server* S = get_server(ctx);
    if (!S) return set_error(RAYPC_ERR_STATE, "no server is running");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return set_error(RAYPC_ERR_INVALID, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
    Request* r = it->second;
    if (r->state == RAYPC_REQ_QUEUED || r->state == RAYPC_REQ_RUNNING) {
        // a cancelled entry may still sit in the queue; the scheduler drops it, so it is safe to keep
        return set_error(RAYPC_ERR_BUSY, "request %llu is not finished", static_cast<unsigned long long>(ticket));
    }
    if (std::find(S->queue.begin(), S->queue.end(), r) != S->queue.end())
        return set_error(RAYPC_ERR_BUSY, "request %llu is still being dropped from the queue",
                         static_cast<unsigned long long>(ticket));
    S->all.erase(it);
    delete r;
    return RAYPC_OK;
}

int raypc_server_get_stats(raypc_ctx* ctx, raypc_server_stats* out) {
    Server* S = get_server(ctx);
    if (!S || !out) return set_error(S ? RAYPC_ERR_INVALID : RAYPC_ERR_STATE, "no server or NULL output");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->inflight = static_cast<int>(S->active.size());
    int queued = 0;
    for (const Request* r : S->queue)
        if (r->state == RAYPC_REQ_QUEUED) ++queued;
    out->queued = queued;
    return RAYPC_OK;
}

}  // extern "C"
