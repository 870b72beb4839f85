// Continuous-batching server for streams of frames from several rigs.
//
// Frames are stateless and independent (one fused cloud per time step, nothing carried
// across frames), so frames of different rigs can share a launch.  The server keeps up to
// `lanes` resident workspaces, each with its own stream.  A scheduler thread admits arrived
// frames into the next free lane as one batch (FIFO by arrival, equal parameters, up to the
// frame and camera limits) launches it with ff_fuse_batch and polls its completion event;
// the next batch can start on another lane while the previous one still runs.
// Latency = completion (observed by the scheduler thread) - arrival.
//
// Admission is by device-memory footprint: the lanes' workspaces together stay within the
// server's budget.  A lane's workspace is sized by the batches it has run (grown when a
// batch needs more, with the budget's consent) or made up front by ff_server_reserve; a
// frame joins a batch only while the batch's workspace fits what the other lanes leave of
// the budget, so a small frame never reserves room for a large one, and a large frame waits
// until room is free (idle lanes give theirs back when the head of the queue does not fit
// anywhere).  The head of the queue prefers a free lane that holds it as it is (the one that
// last ran its rig first, whose graphs for that shape are cached), then an empty lane, then
// the largest other one, since growing a lane re-creates its workspace.
//
// Ordering with the caller: at submit an event is recorded on the caller's stream, and
// the lane waits for it before the frame's batch runs, so work the caller queued before
// the submit (filling the images, clearing the outputs) completes first.
//
// Errors belong to the frame that caused them: a frame the host checks reject is refused
// at submit; a batch whose launch fails completes its own frames with that status, after
// the lane's queued work has finished.  Other frames and later submits are not affected.
//
// The plain baseline (config.plain = 1) runs the same trace one frame at a time through
// ff_fuse and starts a frame only after the previous one completed.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fuseflow.h"
#include "internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    uint64_t ticket;
    int32_t rig;
    double arrival;
    uint64_t pixels;
    std::vector<ff_camera> cams;
    std::vector<ff_view> views;
    ff_params params;
    ff_output out;
    hipEvent_t ready;       // recorded on the caller's stream at submit
};

struct Lane {
    ff_context* ctx = nullptr;
    uint64_t cap_px = 0;          // workspace limits of ctx (0: no workspace)
    int32_t cap_cams = 0, cap_frames = 0;
    uint64_t foot = 0;            // its device bytes
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    bool synced = false;          // the lane's work is known complete (no event to query)
    int32_t last_rig = -1;        // rig of the first frame of its last batch
    ff_status launch_status = FF_OK;
    std::vector<Job> batch;
};

bool same_params(const ff_params& a, const ff_params& b) {
    return std::memcmp(&a, &b, sizeof(ff_params)) == 0;
}

enum TicketPhase : int { kQueued = 0, kRunning = 1, kDone = 2 };

struct TicketState {
    int phase;
    ff_status status;
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct ff_server {
    int device = 0;
    ff_server_config cfg{};
    uint64_t max_px = 0;          // largest single frame the budget admits (pixels)
    uint64_t used = 0, peak = 0;  // bytes of the lanes' workspaces now / at most
    int32_t probe_slot = -1;      // kernel probed in every lane's calls (-1: none)
    ff_probe probe_gone{};        // probe totals of workspaces already given back
    Clock::time_point t0;
    std::vector<Lane> lanes;
    // shared state (mutex)
    std::mutex mu;
    std::condition_variable cv_done;   // frames completed
    std::condition_variable cv_work;   // new submissions
    std::multimap<double, Job> pending;   // by arrival time (ties keep submission order)
    std::unordered_map<uint64_t, TicketState> state;
    std::vector<hipEvent_t> free_events;
    uint64_t next_ticket = 1;
    uint64_t outstanding = 0;
    ff_status drain_status = FF_OK;       // first failure since the last drain
    bool stop = false;
    // stats (mutex)
    std::vector<double> lat_ms;        // completed frames, in completion order
    std::vector<int32_t> lat_rig;      // their rigs
    uint64_t frames = 0, pixels = 0, batches = 0, batch_frames = 0;
    double first_arrival = -1.0, last_done = 0.0;
    std::thread worker;

    double now() const {
        return std::chrono::duration<double>(Clock::now() - t0).count();
    }
    void run();
    bool launch(Lane& L, double t);
    std::vector<Lane*> lane_order(const Job& head);
    void complete(Lane& L, double t, ff_status st);
    bool reserve(Lane& L, uint64_t px, int32_t cams, int32_t frames);
    void release(Lane& L);
};

// Give the lane a workspace for at least (px, cams, frames) if the budget allows; an idle
// lane's old workspace is freed first.  Returns false (nothing changed) when it would not
// fit.
bool ff_server::reserve(Lane& L, uint64_t px, int32_t cams, int32_t frames) {
    if (L.ctx && px <= L.cap_px && cams <= L.cap_cams && frames <= L.cap_frames) return true;
    // grow every limit at least to what is asked, with some headroom for pixels
    const uint64_t npx = std::max<uint64_t>(px, L.cap_px);
    const int32_t nc = std::max(cams, L.cap_cams), nf = std::max(frames, L.cap_frames);
    uint64_t want = npx + npx / 4;
    if (want >= 0xFFFFFFFEull) want = npx;
    uint64_t foot = ff_workspace_bytes(want, nc, nf);
    if (used - L.foot + foot > cfg.hbm_budget_bytes) {
        want = npx;
        foot = ff_workspace_bytes(want, nc, nf);
        if (used - L.foot + foot > cfg.hbm_budget_bytes) return false;
    }
    ff_context* keep = L.ctx;
    if (L.ctx) release(L);
    ff_context* nctx = nullptr;
    if (ff_context_create(&nctx, device, want, nc, nf) != FF_OK) return false;
    if (probe_slot >= 0) (void)ff_probe_enable(nctx, probe_slot);
    if (keep == nullptr) {
        // tunings learnt so far by other lanes
        for (Lane& o : lanes)
            if (o.ctx) { ff::share_tuning(o.ctx, nctx); break; }
    }
    L.ctx = nctx;
    L.cap_px = want;
    L.cap_cams = nc;
    L.cap_frames = nf;
    L.foot = foot;
    used += foot;
    peak = std::max(peak, used);
    for (Lane& o : lanes)
        if (o.ctx && &o != &L) ff::share_tuning(o.ctx, L.ctx);
    return true;
}

// Free an idle lane's workspace (its stream has no queued work).
void ff_server::release(Lane& L) {
    if (!L.ctx) return;
    (void)hipStreamSynchronize(L.stream);
    for (Lane& o : lanes)
        if (o.ctx && &o != &L) ff::share_tuning(L.ctx, o.ctx);
    if (probe_slot >= 0) {
        ff_probe p{};
        if (ff_probe_read(L.ctx, &p) == FF_OK) {
            probe_gone.launches += p.launches;
            probe_gone.frames += p.frames;
            probe_gone.pixels += p.pixels;
            probe_gone.total_ms += p.total_ms;
        }
    }
    ff_context_destroy(L.ctx);
    L.ctx = nullptr;
    used -= L.foot;
    L.foot = 0;
    L.cap_px = 0;
    L.cap_cams = L.cap_frames = 0;
    L.last_rig = -1;
}

// Free lanes in the order the head frame should try them: lanes whose workspace holds it
// as it is (the one that last ran its rig first: its graphs for the rig's shape are
// cached; then the smallest), then lanes without a workspace, then the others, largest
// first (growing a lane frees and re-creates its workspace and captures new graphs).
std::vector<Lane*> ff_server::lane_order(const Job& head) {
    std::vector<Lane*> fit, empty, grow;
    for (Lane& L : lanes) {
        if (L.busy) continue;
        if (!L.ctx) empty.push_back(&L);
        else if (head.pixels <= L.cap_px && (int32_t)head.cams.size() <= L.cap_cams) fit.push_back(&L);
        else grow.push_back(&L);
    }
    std::stable_sort(fit.begin(), fit.end(), [&](const Lane* a, const Lane* b) {
        const bool ra = a->last_rig == head.rig, rb = b->last_rig == head.rig;
        if (ra != rb) return ra;
        return a->foot < b->foot;
    });
    std::stable_sort(grow.begin(), grow.end(),
                     [](const Lane* a, const Lane* b) { return a->foot > b->foot; });
    fit.insert(fit.end(), empty.begin(), empty.end());
    fit.insert(fit.end(), grow.begin(), grow.end());
    return fit;
}

bool ff_server::launch(Lane& L, double t) {
    // caller holds mu; take arrived frames FIFO while the batch's workspace fits this lane,
    // grown as far as the budget the other lanes leave allows
    L.batch.clear();
    uint64_t px = 0, cams = 0;
    const int max_frames = cfg.plain ? 1 : cfg.max_batch_frames;
    const uint64_t room = cfg.hbm_budget_bytes - (used - L.foot);
    auto first = pending.end();
    int nb = 0;
    for (auto it = pending.begin(); it != pending.end() && it->first <= t; ++it) {
        const Job& j = it->second;
        if (nb >= max_frames) break;
        if (nb > 0 && !same_params(j.params, first->second.params)) break;
        if (cams + j.cams.size() > (uint64_t)cfg.max_cameras) break;
        const uint64_t npx = px + j.pixels, nc = cams + j.cams.size();
        const bool fits_now = L.ctx && npx <= L.cap_px && (int32_t)nc <= L.cap_cams &&
                              nb + 1 <= L.cap_frames;
        if (!fits_now &&
            ff_workspace_bytes(std::max<uint64_t>(npx, L.cap_px),
                               std::max<int32_t>((int32_t)nc, L.cap_cams),
                               std::max<int32_t>(nb + 1, L.cap_frames)) > room)
            break;
        if (nb == 0) first = it;
        px = npx;
        cams = nc;
        ++nb;
    }
    if (nb == 0) return false;
    if (!reserve(L, px, (int32_t)cams, nb)) {
        if (used == 0 && L.ctx == nullptr) {
            // nothing else holds device memory and the workspace still cannot be made:
            // the head frame cannot run at all
            auto it = pending.begin();
            L.batch.push_back(std::move(it->second));
            pending.erase(it);
            state[L.batch.back().ticket].phase = kRunning;
            L.synced = true;
            L.launch_status = FF_ERR_OOM;
            L.busy = true;
            return true;
        }
        return false;
    }
    for (int k = 0; k < nb; ++k) {
        auto it = pending.begin();
        state[it->second.ticket].phase = kRunning;
        L.batch.push_back(std::move(it->second));
        pending.erase(it);
    }
    L.last_rig = L.batch.front().rig;
    std::vector<ff_frame> frames(L.batch.size());
    std::vector<ff_output> outs(L.batch.size());
    ff_status st = FF_OK;
    for (size_t i = 0; i < L.batch.size(); ++i) {
        frames[i].n_cams = (int32_t)L.batch[i].cams.size();
        frames[i].cams = L.batch[i].cams.data();
        frames[i].views = L.batch[i].views.data();
        outs[i] = L.batch[i].out;
        // the caller's work queued before the submit comes first
        if (st == FF_OK && hipStreamWaitEvent(L.stream, L.batch[i].ready, 0) != hipSuccess)
            st = FF_ERR_HIP;
    }
    if (st == FF_OK && cfg.autotune && !cfg.plain) {
        // the first batch of a new shape: tune it on this lane, share with the others
        ff_tuning t;
        int32_t found = 0;
        st = ff_tuning_lookup(L.ctx, (int32_t)frames.size(), frames.data(), &L.batch[0].params,
                              &t, &found);
        if (st == FF_OK && !found) {
            st = ff_autotune(L.ctx, (int32_t)frames.size(), frames.data(), &L.batch[0].params,
                             outs.data(), L.stream, &t);
            if (st == FF_OK)
                for (Lane& o : lanes) ff::share_tuning(L.ctx, o.ctx);
        }
    }
    if (st == FF_OK) {
        if (cfg.plain)
            st = ff_fuse(L.ctx, frames[0].n_cams, frames[0].cams, frames[0].views,
                         &L.batch[0].params, &outs[0], L.stream);
        else
            st = ff_fuse_batch(L.ctx, (int32_t)frames.size(), frames.data(),
                               &L.batch[0].params, outs.data(), L.stream);
    }
    // completion is reported once the lane's queued work has finished, also after a
    // failed launch (part of the batch may have been queued)
    if (hipEventRecord(L.done, L.stream) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(L.stream);
        (void)hipGetLastError();
        L.synced = true;
        if (st == FF_OK) st = FF_ERR_HIP;
    }
    L.launch_status = st;
    L.busy = true;
    ++batches;
    batch_frames += L.batch.size();
    return true;
}

void ff_server::complete(Lane& L, double t, ff_status st) {
    for (Job& j : L.batch) {
        TicketState& ts = state[j.ticket];
        ts.phase = kDone;
        ts.status = st;
        if (st != FF_OK && drain_status == FF_OK) drain_status = st;
        free_events.push_back(j.ready);
        if (st == FF_OK) {
            if (first_arrival < 0 || j.arrival < first_arrival) first_arrival = j.arrival;
            lat_ms.push_back((t - j.arrival) * 1e3);
            lat_rig.push_back(j.rig);
            ++frames;
            pixels += j.pixels;
        }
        --outstanding;
    }
    if (st == FF_OK) last_done = std::max(last_done, t);
    L.batch.clear();
    L.busy = false;
    L.synced = false;
    L.launch_status = FF_OK;
}

void ff_server::run() {
    (void)hipSetDevice(device);
    // the scheduler polls running batches every few microseconds: with the kernel's default
    // 50 us timer slack each such sleep would last ~55 us, which delays both the detection of
    // a completed frame and the launch of the next batch on its lane
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        bool progressed = false;
        // 1. completions (event queries are cheap and non-blocking)
        for (Lane& L : lanes) {
            if (!L.busy) continue;
            hipError_t q = L.synced ? hipSuccess : hipEventQuery(L.done);
            if (q == hipSuccess) {
                complete(L, now(), L.launch_status);
                progressed = true;
            } else if (q != hipErrorNotReady) {
                // the event cannot be queried: wait for the lane's work itself before its
                // frames are reported done
                (void)hipGetLastError();
                lk.unlock();
                (void)hipStreamSynchronize(L.stream);
                (void)hipGetLastError();
                lk.lock();
                complete(L, now(), FF_ERR_HIP);
                progressed = true;
            }
        }
        if (progressed) cv_done.notify_all();
        // 2. admissions into free lanes, in the order of preference for the head frame
        const double t = now();
        bool launched = false, idle_free = false;
        while (!pending.empty() && pending.begin()->first <= t) {
            bool any = false;
            for (Lane* L : lane_order(pending.begin()->second))
                if (launch(*L, t)) { any = true; break; }
            if (!any) break;
            progressed = launched = true;
        }
        if (!launched && !pending.empty() && pending.begin()->first <= t) {
            // the head of the queue fits no free lane: idle lanes give their workspaces
            // back (largest first), so that it can be admitted
            Lane* big = nullptr;
            for (Lane& L : lanes)
                if (!L.busy && L.ctx && (!big || L.foot > big->foot)) big = &L;
            if (big) {
                release(*big);
                idle_free = true;
            }
        }
        if (idle_free) continue;
        if (stop && pending.empty() && std::none_of(lanes.begin(), lanes.end(),
                                                    [](const Lane& L) { return L.busy; }))
            break;
        if (progressed) continue;
        const bool any_busy = std::any_of(lanes.begin(), lanes.end(),
                                          [](const Lane& L) { return L.busy; });
        if (any_busy) {
            // a batch is running: poll its event at a few-microsecond granularity
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(5));
            lk.lock();
        } else if (!pending.empty()) {
            const double wait = pending.begin()->first - now();
            if (wait > 2e-4) {
                cv_work.wait_for(lk, std::chrono::duration<double>(wait - 1e-4));
            } else if (wait > 0) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(5));
                lk.lock();
            }
        } else {
            cv_work.wait(lk, [&] { return stop || !pending.empty(); });
        }
    }
}

extern "C" {

void ff_server_config_default(ff_server_config* c) {
    if (!c) return;
    c->hbm_budget_bytes = 16ull << 30;
    c->lanes = 2;
    c->max_batch_frames = 16;
    c->max_cameras = 256;
    c->max_pending = 4096;
    c->plain = 0;
    c->autotune = 0;
}

ff_status ff_server_create(ff_server** out, int device, const ff_server_config* cfg) {
    if (!out || !cfg) return FF_ERR_INVALID_ARG;
    *out = nullptr;
    ff_server_config c = *cfg;
    if (c.plain) { c.lanes = 1; c.max_batch_frames = 1; }
    if (c.lanes < 1 || c.lanes > 8 || c.max_batch_frames < 1 || c.max_batch_frames > 64 ||
        c.max_cameras < 1 || c.max_cameras > 1024 || c.max_pending < 1)
        return FF_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return FF_ERR_INVALID_ARG;
    // largest single frame (pixels, at the camera limit) whose workspace fits the budget
    uint64_t lo = 0, hi = 0xFFFFFFFEull;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (ff_workspace_bytes(mid, c.max_cameras, 1) <= c.hbm_budget_bytes) lo = mid;
        else hi = mid - 1;
    }
    if (lo < 4096) return FF_ERR_OOM;
    ff_server* s = new ff_server();
    s->device = device;
    s->cfg = c;
    s->max_px = lo;
    s->t0 = Clock::now();
    DeviceGuard g(device);
    s->lanes.resize(c.lanes);
    ff_status st = FF_OK;
    for (Lane& L : s->lanes) {
        // workspaces are made when a lane first takes a batch (sized by it)
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
            st = FF_ERR_HIP;
            break;
        }
    }
    if (st != FF_OK) {
        ff_server_destroy(s);
        return st;
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return FF_OK;
}

void ff_server_destroy(ff_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    DeviceGuard g(s->device);
    for (Lane& L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.ctx) ff_context_destroy(L.ctx);
    }
    for (auto& kv : s->pending) s->free_events.push_back(kv.second.ready);
    for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
    delete s;
}

uint64_t ff_server_max_pixels(const ff_server* s) { return s ? s->max_px : 0; }

ff_status ff_server_reserve(ff_server* s, uint64_t pixels, int32_t cameras, int32_t frames) {
    if (!s || pixels == 0 || cameras < 1 || frames < 1 || cameras > s->cfg.max_cameras ||
        frames > (s->cfg.plain ? 1 : s->cfg.max_batch_frames))
        return FF_ERR_INVALID_ARG;
    DeviceGuard g(s->device);
    std::lock_guard<std::mutex> lk(s->mu);
    ff_status st = FF_OK;
    for (Lane& L : s->lanes) {
        if (L.busy) {
            st = FF_ERR_BUSY;
            continue;
        }
        if (!s->reserve(L, pixels, cameras, frames) && st == FF_OK) st = FF_ERR_OOM;
    }
    return st;
}

double ff_server_now(const ff_server* s) { return s ? s->now() : 0.0; }

ff_status ff_server_submit(ff_server* s, int32_t rig_id, const ff_frame* frame,
                           const ff_params* params, const ff_output* out, double arrival_s,
                           void* stream, uint64_t* ticket) {
    if (!s || !frame || !params || !out || !ticket) return FF_ERR_INVALID_ARG;
    // the host checks of the fusion call, for this frame alone
    ff_status st = ff::check_frame(*frame, *params, *out);
    if (st != FF_OK) return st;
    Job j;
    j.rig = rig_id;
    j.cams.assign(frame->cams, frame->cams + frame->n_cams);
    j.views.assign(frame->views, frame->views + frame->n_cams);
    j.params = *params;
    j.out = *out;
    j.pixels = 0;
    for (const ff_camera& c : j.cams) j.pixels += (uint64_t)c.width * (uint64_t)c.height;
    // a frame whose own workspace exceeds the whole budget can never be admitted
    if (j.cams.size() > (size_t)s->cfg.max_cameras ||
        ff_workspace_bytes(j.pixels, (int32_t)j.cams.size(), 1) > s->cfg.hbm_budget_bytes)
        return FF_ERR_OOM;
    DeviceGuard g(s->device);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->pending.size() >= (size_t)s->cfg.max_pending) return FF_ERR_BUSY;
        if (s->free_events.empty()) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return FF_ERR_HIP;
            }
            s->free_events.push_back(e);
        }
        j.ready = s->free_events.back();
        if (hipEventRecord(j.ready, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
            (void)hipGetLastError();
            return FF_ERR_HIP;
        }
        s->free_events.pop_back();
        j.ticket = s->next_ticket++;
        // an arrival in the past (or none given) is the moment of this call
        j.arrival = std::max(arrival_s, s->now());
        *ticket = j.ticket;
        s->state[j.ticket] = TicketState{kQueued, FF_OK};
        ++s->outstanding;
        const double a = j.arrival;
        s->pending.emplace(a, std::move(j));
    }
    s->cv_work.notify_all();
    return FF_OK;
}

ff_status ff_server_poll(ff_server* s, uint64_t ticket, int32_t* done) {
    if (!s || !done) return FF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->state.find(ticket);
    if (it == s->state.end()) return FF_ERR_NOT_FOUND;
    *done = it->second.phase == kDone ? 1 : 0;
    if (!*done) return FF_OK;
    const ff_status st = it->second.status;
    s->state.erase(it);
    return st;
}

ff_status ff_server_wait(ff_server* s, uint64_t ticket) {
    if (!s) return FF_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->state.find(ticket);
    if (it == s->state.end()) return FF_ERR_NOT_FOUND;
    s->cv_done.wait(lk, [&] {
        auto f = s->state.find(ticket);
        return f == s->state.end() || f->second.phase == kDone;
    });
    it = s->state.find(ticket);
    if (it == s->state.end()) return FF_ERR_NOT_FOUND;   // reported by a concurrent call
    const ff_status st = it->second.status;
    s->state.erase(it);
    return st;
}

ff_status ff_server_drain(ff_server* s) {
    if (!s) return FF_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
    // every ticket is done: their statuses are reported here, once
    s->state.clear();
    const ff_status st = s->drain_status;
    s->drain_status = FF_OK;
    return st;
}

ff_status ff_server_stats(const ff_server* cs, ff_stats* st) {
    if (!cs || !st) return FF_ERR_INVALID_ARG;
    ff_server* s = const_cast<ff_server*>(cs);
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof(*st));
    st->frames = s->frames;
    st->pixels = s->pixels;
    st->batches = s->batches;
    st->first_arrival_s = s->first_arrival;
    st->last_done_s = s->last_done;
    st->mean_batch_frames = s->batches ? (double)s->batch_frames / (double)s->batches : 0.0;
    st->hbm_used_bytes = s->used;
    st->hbm_peak_bytes = s->peak;
    if (!s->lat_ms.empty()) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(q * v.size()) - 1);
            return v[i];
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        st->max_ms = v.back();
        double sum = 0;
        for (double x : v) sum += x;
        st->mean_ms = sum / v.size();
        const double span = s->last_done - s->first_arrival;
        st->px_per_s = span > 0 ? (double)s->pixels / span : 0.0;
    }
    return FF_OK;
}

ff_status ff_server_latencies(const ff_server* cs, uint64_t cap, int32_t* rig_ids,
                              double* latency_ms, uint64_t* n) {
    if (!cs || !n) return FF_ERR_INVALID_ARG;
    ff_server* s = const_cast<ff_server*>(cs);
    std::lock_guard<std::mutex> lk(s->mu);
    *n = s->lat_ms.size();
    const size_t k = (size_t)std::min<uint64_t>(cap, s->lat_ms.size());
    for (size_t i = 0; i < k; ++i) {
        if (rig_ids) rig_ids[i] = s->lat_rig[i];
        if (latency_ms) latency_ms[i] = s->lat_ms[i];
    }
    return FF_OK;
}

ff_status ff_server_reset_stats(ff_server* s) {
    if (!s) return FF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    s->lat_ms.clear();
    s->lat_rig.clear();
    s->frames = s->pixels = s->batches = s->batch_frames = 0;
    s->first_arrival = -1.0;
    s->last_done = 0.0;
    return FF_OK;
}

ff_status ff_server_probe_enable(ff_server* s, int32_t slot) {
    if (!s || slot < -1 || slot >= FF_TRACE_SLOTS) return FF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);    // the scheduler launches under this lock
    ff_status st = FF_OK;
    s->probe_slot = slot;
    s->probe_gone = ff_probe{};
    for (Lane& L : s->lanes) {
        if (!L.ctx) continue;
        const ff_status e = ff_probe_enable(L.ctx, slot);
        if (e != FF_OK) st = e;
    }
    return st;
}

ff_status ff_server_probe_read(ff_server* s, ff_probe* out) {
    if (!s || !out) return FF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->slot = s->probe_slot;
    out->launches = s->probe_gone.launches;
    out->frames = s->probe_gone.frames;
    out->pixels = s->probe_gone.pixels;
    out->total_ms = s->probe_gone.total_ms;
    ff_status st = FF_OK;
    for (Lane& L : s->lanes) {
        if (!L.ctx) continue;
        ff_probe p{};
        const ff_status e = ff_probe_read(L.ctx, &p);
        if (e != FF_OK) st = e;
        out->slot = p.slot;
        out->launches += p.launches;
        out->frames += p.frames;
        out->pixels += p.pixels;
        out->total_ms += p.total_ms;
    }
    return st;
}

}  // extern "C"
