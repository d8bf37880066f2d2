// Served stream: continuous batching of frames over launch lanes.
//
// Submitted frames wait in arrival order. A host dispatcher thread owns a few
// lanes, each a stream with at most one launch of the persistent filter
// kernel in flight. Whenever a lane is free it takes the waiting frames, in
// arrival order, whose scratch (bit planes and level entries) still fits in
// the server's device pool -- admission by HBM footprint -- up to a per-launch
// cap, and launches them as one cost-ordered batch. Frames that arrive while
// other launches run go into the next free lane, so their work overlaps on
// the device with the frames already there. The kernel sets a completion word
// in host-mapped memory after each frame, so a frame is handed out, and its
// scratch returned to the pool, as soon as it is done, not when its launch
// ends. A frame of at least the context's batch_grid_min_pixels pixels is
// launched alone, filtered by a grid of workgroups, and completes with its
// launch.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hasf_common.h"

namespace hasf_detail {
hipError_t launch_filter(const ImgDesc* d_desc, int n, int* d_next, int grid, int block, size_t lds_bytes,
                         hipStream_t stream, unsigned* done);
int filter_occupancy(size_t lds_bytes, int block);
int filter_block_for(int n, int num_cu);
hipError_t launch_grid(const ImgDesc* d_desc, GridCtl* d_ctl, unsigned* d_err, int grid, hipStream_t stream);
int grid_occupancy();
void record_error(hasf_ctx* ctx, const char* msg);
}  // namespace hasf_detail

using namespace hasf_detail;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// first-fit allocator over [0, size) in 256-byte units
struct Pool {
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size = 0, used = 0, peak = 0;

    void init(size_t n)
    {
        size = n;
        free_.clear();
        if (n)
            free_[0] = n;
        used = peak = 0;
    }
    bool alloc(size_t n, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t at = it->first + n;
                free_.erase(it);
                if (rest)
                    free_[at] = rest;
                used += n;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Frame {
    uint64_t ticket = 0;
    hasf_image img{};   // as the kernel reads it (device pointers)
    hasf_image himg{};  // a host frame: the caller's host buffers
    bool host = false;  // copied to pool memory before its launch and back after it
    size_t stage_bytes = 0;  // host frames: X, C and D packed (pitch W) after the scratch
    ImageLayout lay{};
    double cost = 0;
    bool grid = false;  // filtered by a grid of workgroups, alone in its launch
    size_t off = 0;     // pool offset in bytes
    double t_submit = 0, t_done = 0;
    int status = HASF_OK;
    bool done = false;
};

// one stream with at most one launch in flight
struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    char* d_meta = nullptr;      // device: [queue counter | descriptors], or [GridCtl | descriptor]
    char* h_meta = nullptr;      // pinned staging of d_meta
    unsigned* h_done = nullptr;  // host-mapped completion words, one per queue position
    unsigned* d_done = nullptr;  // the same words as the kernel addresses them
    std::vector<Frame*> frames;  // queue position -> frame (nullptr once retired)
    bool busy = false;
    bool grid = false;           // the launch is one grid frame
    bool express = false;        // takes only small frames
};

// offset of the descriptor after a GridCtl in a lane's meta block
constexpr size_t GRID_DESC_OFF = (sizeof(GridCtl) + 255) / 256 * 256;

// pool bytes of a frame: its scratch, then (host frames) its staged buffers
size_t frame_bytes(const Frame* f)
{
    return f->lay.total() + f->stage_bytes;
}

double frame_cost(const hasf_image& im)
{
    double lv = 0;
    for (int i = 1; i <= im.r; ++i)
        lv += hasf_levels(i) + 1;
    return (double)im.H * im.W * (lv + 1);
}

}  // namespace

struct hasf_server {
    hasf_ctx* ctx = nullptr;
    char* pool_mem = nullptr;
    Pool pool;
    std::vector<Lane> lanes;
    int max_batch = 0;
    int max_pending = 0;
    size_t lds_cap = 0;
    size_t small_px = 0;  // frames of at most this many pixels are small
    bool express = false; // some lanes are express lanes

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Frame*> pending;
    size_t in_flight = 0;
    std::unordered_map<uint64_t, Frame*> frames;
    uint64_t next_ticket = 1;
    bool stopping = false;
    int fatal = HASF_OK;
    char err[256] = "";
    std::thread worker;

    // stats
    uint64_t submitted = 0, completed = 0, rejected = 0, launches = 0, launched_frames = 0;
    int batch_max = 0;
    double t_first = 0, t_last = 0, px_done = 0;
    std::vector<double> lat_ms;
};

namespace {

void retire(hasf_server* s, Frame* f, double t, int status)
{
    f->t_done = t;
    f->status = status;
    f->done = true;
    s->pool.release(f->off / 256, frame_bytes(f) / 256);
    --s->in_flight;
    if (status == HASF_OK) {
        ++s->completed;
        s->t_last = t;
        s->px_done += (double)f->img.H * f->img.W;
        s->lat_ms.push_back((t - f->t_submit) * 1e3);
    }
}

void fill_desc(hasf_server* s, const Frame* f, ImgDesc& d)
{
    d.X = f->img.X;
    d.C = f->img.C;
    d.ld = f->img.ld;
    d.H = f->img.H;
    d.W = f->img.W;
    d.r = f->img.r;
    d.lds = f->lay.lds ? 1 : 0;
    d.D = f->img.D;
    d.conn4 = f->img.conn == 4 ? 1 : 0;
    d.order = f->img.order;
    char* base = s->pool_mem + f->off;
    d.gplanes = (uint64_t*)base;
    d.ent_idx = (uint32_t*)(base + f->lay.planes_bytes);
    d.ent_msk = (uint64_t*)(base + f->lay.planes_bytes + f->lay.idx_bytes);
}

// A host frame's device copies, in its pool block after the scratch: X, C and
// D at pitch W, each 256-byte aligned; img points there from its admission on.
void stage_frame(hasf_server* s, Frame* f)
{
    char* p = s->pool_mem + f->off + f->lay.total();
    const size_t plane = hasf_align256((size_t)f->himg.H * (size_t)f->himg.W);
    f->img = f->himg;
    f->img.ld = f->himg.W;
    f->img.X = (uint8_t*)p;
    f->img.C = f->himg.C ? (const uint8_t*)(p + plane) : nullptr;
    f->img.D = f->himg.D ? (const uint8_t*)(p + (f->himg.C ? 2 : 1) * plane) : nullptr;
}

// the copies in before a launch and of X out after it, on the lane's stream
hipError_t copy_in(const Frame* f, hipStream_t st)
{
    const hasf_image& h = f->himg;
    hipError_t e = hipMemcpy2DAsync(f->img.X, (size_t)h.W, h.X, (size_t)h.ld, (size_t)h.W, (size_t)h.H,
                                    hipMemcpyHostToDevice, st);
    if (e == hipSuccess && h.C)
        e = hipMemcpy2DAsync((void*)f->img.C, (size_t)h.W, h.C, (size_t)h.ld, (size_t)h.W, (size_t)h.H,
                             hipMemcpyHostToDevice, st);
    if (e == hipSuccess && h.D)
        e = hipMemcpy2DAsync((void*)f->img.D, (size_t)h.W, h.D, (size_t)h.ld, (size_t)h.W, (size_t)h.H,
                             hipMemcpyHostToDevice, st);
    return e;
}

hipError_t copy_out(const Frame* f, hipStream_t st)
{
    const hasf_image& h = f->himg;
    return hipMemcpy2DAsync(h.X, (size_t)h.ld, f->img.X, (size_t)h.W, (size_t)h.W, (size_t)h.H,
                            hipMemcpyDeviceToHost, st);
}

void launch_failed(hasf_server* s, hipError_t e)
{
    (void)hipGetLastError();
    s->fatal = HASF_EDEVICE;
    snprintf(s->err, sizeof s->err, "serve launch: %s", hipGetErrorString(e));
}

// A grid frame at the head of the queue: launched alone on `ln`.
bool launch_grid_frame(hasf_server* s, Lane& ln)
{
    Frame* f = s->pending.front();
    size_t off = 0;
    if (!s->pool.alloc(frame_bytes(f) / 256, &off))
        return false;
    f->off = off * 256;
    s->pending.pop_front();
    if (f->host)
        stage_frame(s, f);
    std::memset(ln.h_meta, 0, GRID_DESC_OFF);  // the GridCtl starts at 0
    fill_desc(s, f, *(ImgDesc*)(ln.h_meta + GRID_DESC_OFF));
    ln.h_done[0] = 0;  // not written by the grid kernel; the frame completes with its launch
    ln.frames.assign(1, f);
    ln.busy = true;
    ln.grid = true;
    s->in_flight += 1;
    ++s->launches;
    s->launched_frames += 1;
    s->batch_max = std::max(s->batch_max, 1);
    const int nwd = f->img.H * ((f->img.W + 63) / 64);
    const int grid = grid_blocks(nwd, s->ctx->num_cu * grid_occupancy() / 2);
    hipError_t e = f->host ? copy_in(f, ln.stream) : hipSuccess;
    if (e == hipSuccess)
        e = hipMemcpyAsync(ln.d_meta, ln.h_meta, GRID_DESC_OFF + sizeof(ImgDesc), hipMemcpyHostToDevice, ln.stream);
    if (e == hipSuccess)
        e = launch_grid((const ImgDesc*)(ln.d_meta + GRID_DESC_OFF), (GridCtl*)ln.d_meta, nullptr, grid, ln.stream);
    if (e == hipSuccess && f->host)
        e = copy_out(f, ln.stream);
    if (e == hipSuccess)
        e = hipEventRecord(ln.ev, ln.stream);
    if (e != hipSuccess)
        launch_failed(s, e);
    return true;
}

bool is_small(const hasf_server* s, const Frame* f)
{
    return !f->grid && (size_t)f->img.H * (size_t)f->img.W <= s->small_px;
}

// Launches the waiting frames that fit on `ln`; false if none fits now.
// A launch ends only when its slowest frame is done, so with express lanes a
// launch never mixes small and large frames: a normal lane takes frames in
// arrival order while they are of the head's size class; an express lane
// takes only small frames, in arrival order, passing over the large ones.
// Without express lanes a launch takes the waiting frames in arrival order
// whatever their sizes (each frame is still handed out on its own completion
// word).
bool launch_lane(hasf_server* s, Lane& ln)
{
    if (!ln.express && !s->pending.empty() && s->pending.front()->grid)
        return launch_grid_frame(s, ln);
    std::vector<Frame*> take;
    if (ln.express) {
        for (auto it = s->pending.begin(); it != s->pending.end() && (int)take.size() < s->max_batch;) {
            Frame* f = *it;
            if (!is_small(s, f)) {
                ++it;
                continue;
            }
            size_t off = 0;
            if (!s->pool.alloc(frame_bytes(f) / 256, &off))
                break;  // HBM footprint: wait until frames on the device finish
            f->off = off * 256;
            it = s->pending.erase(it);
            take.push_back(f);
        }
    } else {
        const bool small = !s->pending.empty() && is_small(s, s->pending.front());
        while (!s->pending.empty() && (int)take.size() < s->max_batch) {
            Frame* f = s->pending.front();
            if (f->grid || (s->express && is_small(s, f) != small))
                break;  // alone, or another class: the next free lane takes it
            size_t off = 0;
            if (!s->pool.alloc(frame_bytes(f) / 256, &off))
                break;  // HBM footprint: wait until frames on the device finish
            f->off = off * 256;
            s->pending.pop_front();
            take.push_back(f);
        }
    }
    if (take.empty())
        return false;
    // queue order of the launch: decreasing cost (largest first)
    std::stable_sort(take.begin(), take.end(), [](const Frame* a, const Frame* b) { return a->cost > b->cost; });
    const int n = (int)take.size();
    ImgDesc* desc = (ImgDesc*)(ln.h_meta + 256);
    size_t lds_need = 0;
    bool any_host = false;
    for (int q = 0; q < n; ++q) {
        if (take[q]->host) {
            stage_frame(s, take[q]);
            any_host = true;
        }
        fill_desc(s, take[q], desc[q]);
        lds_need = std::max(lds_need, take[q]->lay.lds_bytes);
        ln.h_done[q] = 0;
    }
    std::memset(ln.h_meta, 0, 256);  // the launch's queue counter starts at 0
    ln.frames = take;
    ln.busy = true;
    ln.grid = false;
    s->in_flight += n;
    ++s->launches;
    s->launched_frames += n;
    s->batch_max = std::max(s->batch_max, n);

    // the lanes share the device: count every frame in flight (this launch's
    // included) against the CUs
    const int block = filter_block_for((int)std::min<uint64_t>(s->in_flight, INT32_MAX), s->ctx->num_cu);
    const int occ = std::max(1, filter_occupancy(lds_need, block));
    const int grid = std::min(n, s->ctx->num_cu * occ);
    // h_meta is pinned and not rewritten before this lane's launch has ended,
    // so the copy may run after this call returns
    hipError_t e = hipSuccess;
    for (int q = 0; q < n && e == hipSuccess && any_host; ++q)
        if (take[q]->host)
            e = copy_in(take[q], ln.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ln.d_meta, ln.h_meta, 256 + sizeof(ImgDesc) * (size_t)n, hipMemcpyHostToDevice,
                           ln.stream);
    if (e == hipSuccess)
        e = launch_filter((const ImgDesc*)(ln.d_meta + 256), n, (int*)ln.d_meta, grid, block, lds_need,
                          ln.stream, ln.d_done);
    // host frames: their results go back after the launch and they complete
    // with it (their completion words only say that the kernel is done)
    for (int q = 0; q < n && e == hipSuccess && any_host; ++q)
        if (take[q]->host)
            e = copy_out(take[q], ln.stream);
    if (e == hipSuccess)
        e = hipEventRecord(ln.ev, ln.stream);
    if (e != hipSuccess)
        launch_failed(s, e);
    return true;
}

void serve_loop(hasf_server* s)
{
    hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        // retire: frames whose completion word is set, then ended launches
        for (Lane& ln : s->lanes) {
            if (!ln.busy)
                continue;
            const double t = now_s();
            for (size_t q = 0; q < ln.frames.size() && !ln.grid; ++q) {
                Frame* f = ln.frames[q];
                if (f && !f->host && __atomic_load_n(ln.h_done + q, __ATOMIC_ACQUIRE)) {
                    retire(s, f, t, HASF_OK);
                    ln.frames[q] = nullptr;
                    progress = true;
                }
            }
            const hipError_t e = hipEventQuery(ln.ev);
            if (e == hipErrorNotReady)
                continue;
            if (e != hipSuccess) {
                (void)hipGetLastError();
                if (s->fatal == HASF_OK) {
                    s->fatal = HASF_EDEVICE;
                    snprintf(s->err, sizeof s->err, "serve kernel: %s", hipGetErrorString(e));
                }
            }
            // the launch has ended: a frame without its completion word failed;
            // a grid frame failed if its barrier gave up
            const double t2 = now_s();
            bool grid_ok = true;
            if (ln.grid && e == hipSuccess) {
                unsigned gerr = 1;
                hipError_t ec = hipMemcpyAsync(&gerr, ln.d_meta + offsetof(GridCtl, err), sizeof gerr,
                                               hipMemcpyDeviceToHost, ln.stream);
                if (ec == hipSuccess)
                    ec = hipStreamSynchronize(ln.stream);
                grid_ok = ec == hipSuccess && gerr == 0;
                if (ec != hipSuccess)
                    (void)hipGetLastError();
            }
            for (size_t q = 0; q < ln.frames.size(); ++q) {
                if (Frame* f = ln.frames[q]) {
                    const bool ok = e == hipSuccess && (ln.grid ? grid_ok : __atomic_load_n(ln.h_done + q, __ATOMIC_ACQUIRE) != 0);
                    retire(s, f, t2, ok ? HASF_OK : (e == hipSuccess ? HASF_EINTERNAL : HASF_EDEVICE));
                }
            }
            ln.frames.clear();
            ln.busy = false;
            progress = true;
        }
        // launch waiting frames on free lanes
        if (s->fatal == HASF_OK) {
            for (Lane& ln : s->lanes) {
                if (s->pending.empty())
                    break;
                if (!ln.busy && launch_lane(s, ln))
                    progress = true;
            }
        } else if (!s->pending.empty()) {
            const double t = now_s();
            for (Frame* f : s->pending) {
                f->status = s->fatal;
                f->t_done = t;
                f->done = true;
            }
            s->pending.clear();
            progress = true;
        }
        if (progress)
            s->cv_done.notify_all();
        if (s->stopping && s->pending.empty() && s->in_flight == 0)
            break;
        if (s->pending.empty() && s->in_flight == 0) {
            s->cv_work.wait(lk);
        } else {
            // frames on the device: poll their completion words
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(progress ? 2 : 10));
            lk.lock();
        }
    }
}

void free_server(hasf_server* s)
{
    for (Lane& ln : s->lanes) {
        if (ln.ev)
            hipEventDestroy(ln.ev);
        if (ln.stream)
            hipStreamDestroy(ln.stream);
        if (ln.d_meta)
            hipFree(ln.d_meta);
        if (ln.h_meta)
            hipHostFree(ln.h_meta);
        if (ln.h_done)
            hipHostFree(ln.h_done);
    }
    if (s->pool_mem)
        hipFree(s->pool_mem);
    for (auto& kv : s->frames)
        delete kv.second;
    delete s;
}

}  // namespace

extern "C" {

// Lanes by default: one per hardware queue the HIP runtime gives the process
// (GPU_MAX_HW_QUEUES, 4 when unset). Launches on streams beyond the hardware
// queues share a queue and run one after the other, so more lanes than
// queues add nothing.
static int default_lanes()
{
    int q = 4;
    if (const char* v = std::getenv("GPU_MAX_HW_QUEUES")) {
        const int n = std::atoi(v);
        if (n > 0)
            q = n;
    }
    return std::max(1, std::min(q, (int)HASF_SERVE_LANES_MAX));
}

hasf_status hasf_serve(hasf_ctx* ctx, const hasf_serve_opts* opts, hasf_server** out)
{
    if (!ctx || !out) {
        record_error(ctx, "hasf_serve: ctx and out must not be NULL");
        return HASF_EINVAL;
    }
    *out = nullptr;
    hasf_serve_opts o{};
    if (opts)
        o = *opts;
    if (o.flags & HASF_SERVE_PERSISTENT) {
        record_error(ctx, "hasf_serve: the persistent polling kernel (HASF_SERVE_PERSISTENT) is switched off");
        return HASF_EINTERNAL;
    }
    if (o.flags != 0 || o.lanes < 0 || o.lanes > HASF_SERVE_LANES_MAX || o.max_batch < 0 || o.max_pending < 0 ||
        o.express_lanes < -1 || o.express_max_pixels < 0) {
        record_error(ctx, "hasf_serve: bad options");
        return HASF_EINVAL;
    }
    const int nlanes = o.lanes ? o.lanes : default_lanes();
    // default: 3/8 of the lanes (6 of 16: on the mixed 2000 frames/s stream of
    // sides 256..2048 on MI355X, frames of at most 0.5 Mpx waited p99 7.5 ms
    // with 6 express lanes of 16, 23 ms with 5, 35 ms with 4, 41 ms with
    // none, the overall rate unchanged)
    const int nexpress = o.express_lanes < 0 ? std::max(1, nlanes * 3 / 8) : o.express_lanes;
    if (nexpress >= nlanes && !(o.express_lanes < 0 && nlanes == 1)) {
        record_error(ctx, "hasf_serve: express_lanes must be fewer than the lanes");
        return HASF_EINVAL;
    }
    hasf_server* s = new (std::nothrow) hasf_server();
    if (!s)
        return HASF_ENOMEM;
    s->ctx = ctx;
    s->max_batch = o.max_batch ? o.max_batch : 1024;
    s->max_pending = o.max_pending ? o.max_pending : (1 << 20);
    const size_t pool_bytes = (o.pool_bytes ? o.pool_bytes : ctx->hbm_budget) / 256 * 256;
    s->lds_cap = std::min(ctx->lds_per_block, (size_t)160 * 1024) - 2048;
    s->small_px = o.express_max_pixels ? (size_t)o.express_max_pixels : ((size_t)1 << 19);
    s->lanes.resize(nlanes);
    // the last lanes are the express ones (none with a single lane)
    for (int k = 0; k < nlanes; ++k)
        s->lanes[k].express = nlanes > 1 && k >= nlanes - nexpress;
    s->express = nlanes > 1 && nexpress > 0;
    hipSetDevice(ctx->device);
    hipError_t e = hipMalloc((void**)&s->pool_mem, std::max(pool_bytes, (size_t)256));
    const size_t meta = std::max(256 + sizeof(ImgDesc) * (size_t)s->max_batch, GRID_DESC_OFF + sizeof(ImgDesc));
    for (Lane& ln : s->lanes) {
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipMalloc((void**)&ln.d_meta, meta);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&ln.h_meta, meta, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&ln.h_done, sizeof(unsigned) * (size_t)s->max_batch,
                              hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess)
            e = hipHostGetDevicePointer((void**)&ln.d_done, ln.h_done, 0);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        char msg[256];
        snprintf(msg, sizeof msg, "hasf_serve: %s", hipGetErrorString(e));
        record_error(ctx, msg);
        const hasf_status st = e == hipErrorOutOfMemory ? HASF_ENOMEM : HASF_EDEVICE;
        free_server(s);
        return st;
    }
    s->pool.init(pool_bytes / 256);
    s->worker = std::thread(serve_loop, s);
    *out = s;
    return HASF_OK;
}

namespace {

hasf_status submit(hasf_server* s, const hasf_image* img, uint64_t* ticket, bool host)
{
    if (!s || !img || !ticket)
        return HASF_EINVAL;
    if (!img->X || img->H < 1 || img->W < 1 || (int64_t)img->H + img->W > 65535 || img->ld < img->W ||
        img->r < 0 || img->r > HASF_R_MAX || (img->conn != 0 && img->conn != 4 && img->conn != 8) ||
        (img->order != 0 && img->order != 1)) {
        std::lock_guard<std::mutex> g(s->mu);
        ++s->rejected;
        return HASF_EINVAL;
    }
    Frame* f = new (std::nothrow) Frame();
    if (!f)
        return HASF_ENOMEM;
    f->img = *img;
    if (host) {
        f->host = true;
        f->himg = *img;
        f->stage_bytes = hasf_align256((size_t)img->H * (size_t)img->W) * (1 + (img->C ? 1 : 0) + (img->D ? 1 : 0));
    }
    f->grid = (size_t)img->H * (size_t)img->W >= s->ctx->batch_grid_min_px;
    f->lay = image_layout(img->H, img->W, img->r, f->grid ? 0 : s->lds_cap);
    f->cost = frame_cost(*img);
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stopping || s->fatal != HASF_OK) {
            delete f;
            return s->fatal != HASF_OK ? (hasf_status)s->fatal : HASF_EINVAL;
        }
        if (frame_bytes(f) > s->pool.size * 256) {
            ++s->rejected;
            delete f;
            return HASF_ENOMEM;  // could never be admitted
        }
        if ((int)s->pending.size() >= s->max_pending) {
            delete f;
            return HASF_EAGAIN;
        }
        f->ticket = s->next_ticket++;
        f->t_submit = now_s();
        if (s->submitted == 0)
            s->t_first = f->t_submit;
        ++s->submitted;
        s->frames[f->ticket] = f;
        s->pending.push_back(f);
        *ticket = f->ticket;
    }
    s->cv_work.notify_one();
    return HASF_OK;
}

}  // namespace

hasf_status hasf_serve_submit(hasf_server* s, const hasf_image* img, uint64_t* ticket)
{
    return submit(s, img, ticket, false);
}

hasf_status hasf_serve_submit_host(hasf_server* s, const hasf_image* img, uint64_t* ticket)
{
    return submit(s, img, ticket, true);
}

hasf_status hasf_serve_wait(hasf_server* s, uint64_t ticket, int timeout_ms, hasf_result* out)
{
    if (!s)
        return HASF_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->frames.find(ticket);
    if (it == s->frames.end())
        return HASF_EINVAL;
    Frame* f = it->second;
    auto ready = [&] { return f->done; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
        return HASF_ETIMEDOUT;
    }
    if (out) {
        out->status = f->status;
        out->ticket = f->ticket;
        out->submit_s = f->t_submit;
        out->done_s = f->t_done;
        out->latency_ms = (f->t_done - f->t_submit) * 1e3;
    }
    const int st = f->status;
    s->frames.erase(it);
    delete f;
    return (hasf_status)st;
}

hasf_status hasf_serve_stats(hasf_server* s, hasf_stats* out)
{
    if (!s || !out)
        return HASF_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rejected = s->rejected;
    out->pending = s->pending.size();
    out->in_flight = s->in_flight;
    if (!s->lat_ms.empty()) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t k = (size_t)std::min<double>((double)v.size() - 1, std::max(0.0, p * (v.size() - 1) + 0.5));
            return v[k];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = v.back();
        const double span = s->t_last - s->t_first;
        if (span > 0) {
            out->frames_per_s = s->completed / span;
            out->mpixel_per_s = s->px_done / span / 1e6;
        }
    }
    out->pool_bytes = s->pool.size * 256;
    out->pool_peak_bytes = s->pool.peak * 256;
    out->kernel_launches = s->launches;
    out->frames_per_launch = s->launches ? (double)s->launched_frames / (double)s->launches : 0.0;
    out->batch_max = (uint64_t)s->batch_max;
    return HASF_OK;
}

hasf_status hasf_serve_stop(hasf_server* s)
{
    if (!s)
        return HASF_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_one();
    if (s->worker.joinable())
        s->worker.join();
    hipSetDevice(s->ctx->device);
    hipError_t e = hipSuccess;
    for (Lane& ln : s->lanes) {
        const hipError_t el = hipStreamSynchronize(ln.stream);
        if (e == hipSuccess)
            e = el;
    }
    const int fatal = s->fatal;
    if (fatal != HASF_OK)
        record_error(s->ctx, s->err);
    free_server(s);
    if (e != hipSuccess)
        return HASF_EDEVICE;
    return fatal == HASF_OK ? HASF_OK : (hasf_status)fatal;
}

}  // extern "C"
