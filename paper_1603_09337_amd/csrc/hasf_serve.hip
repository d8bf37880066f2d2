// Served stream: host dispatcher of the persistent filter kernel.
//
// Submitted frames wait in arrival order until their scratch fits in the
// server's device pool (admission by HBM footprint) and a ring slot is free;
// the dispatcher then writes the frame's descriptor into a ring in pinned
// host memory and advances the published count, which the kernel's idle
// workgroups poll. A workgroup that finishes a frame stores the frame's
// sequence number in the slot's completion word; the dispatcher sees it,
// stamps the completion time, frees the scratch and wakes waiters. The kernel
// exits when stopped or after an idle period; the dispatcher relaunches it
// whenever published frames are outstanding and it is not running.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
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
hipError_t launch_serve(const ImgDesc* ring, const unsigned long long* tail, const int* stop, int* done,
                        unsigned long long* head, ImgDesc* dev_desc, int cap, unsigned long long idle_limit,
                        int grid, size_t lds_bytes, hipStream_t stream);
int serve_occupancy(size_t lds_bytes);
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
    uint64_t ticket;
    hasf_image img;
    ImageLayout lay;
    size_t off = 0;
    int slot = -1;
    unsigned long long seq = 0;
    double t_submit = 0, t_done = 0;
    int status = HASF_OK;
    bool done = false;
};

}  // namespace

struct hasf_server {
    hasf_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    // pinned host memory (mapped)
    ImgDesc* ring = nullptr;
    unsigned long long* tail = nullptr;
    int* stop = nullptr;
    int* done = nullptr;
    // device pointers of the pinned memory
    ImgDesc* d_ring = nullptr;
    unsigned long long* d_tail = nullptr;
    int* d_stop = nullptr;
    int* d_done = nullptr;
    // device memory
    unsigned long long* head = nullptr;
    ImgDesc* dev_desc = nullptr;
    char* pool_mem = nullptr;
    Pool pool;
    int cap = 0;
    int max_pending = 0;
    unsigned long long idle_ticks = 0;
    size_t lds_cap = 0, lds_launch = 0;
    int grid = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Frame*> pending;
    std::vector<Frame*> inflight;
    std::vector<Frame*> slot_frame;
    std::unordered_map<uint64_t, Frame*> frames;
    uint64_t next_ticket = 1;
    unsigned long long published = 0;
    bool stopping = false;
    bool kernel_running = false;
    int fatal = HASF_OK;
    char err[256] = "";
    std::thread worker;

    // stats
    uint64_t submitted = 0, completed = 0, rejected = 0, launches = 0;
    double t_first = 0, t_last = 0, px_done = 0;
    std::vector<double> lat_ms;
};

namespace {

void serve_loop(hasf_server* s)
{
    hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        // admit in arrival order while memory and ring slots allow
        while (!s->pending.empty() && s->fatal == HASF_OK) {
            Frame* f = s->pending.front();
            const int slot = (int)(s->published % (unsigned long long)s->cap);
            if (s->slot_frame[slot])
                break;  // ring full
            size_t off = 0;
            if (!s->pool.alloc(f->lay.total() / 256, &off))
                break;  // HBM budget: wait for frames to complete
            off *= 256;
            s->pending.pop_front();
            f->off = off;
            f->slot = slot;
            f->seq = s->published;
            ImgDesc d;
            d.X = f->img.X;
            d.C = f->img.C;
            d.ld = f->img.ld;
            d.H = f->img.H;
            d.W = f->img.W;
            d.r = f->img.r;
            d.lds = f->lay.lds ? 1 : 0;
            char* base = s->pool_mem + off;
            d.gplanes = (uint64_t*)base;
            d.ent_idx = (uint32_t*)(base + f->lay.planes_bytes);
            d.ent_msk = (uint64_t*)(base + f->lay.planes_bytes + f->lay.idx_bytes);
            std::memcpy((void*)(s->ring + slot), &d, sizeof d);
            __atomic_store_n(s->done + slot, 0, __ATOMIC_RELAXED);
            s->slot_frame[slot] = f;
            s->inflight.push_back(f);
            ++s->published;
            __atomic_store_n(s->tail, s->published, __ATOMIC_RELEASE);
            progress = true;
        }
        // (re)start the kernel when published frames are outstanding
        if (!s->inflight.empty() && s->fatal == HASF_OK) {
            if (s->kernel_running && hipStreamQuery(s->stream) == hipSuccess)
                s->kernel_running = false;
            if (!s->kernel_running) {
                hipError_t e = launch_serve(s->d_ring, s->d_tail, s->d_stop, s->d_done, s->head, s->dev_desc, s->cap,
                                            s->idle_ticks, s->grid, s->lds_launch, s->stream);
                if (e != hipSuccess) {
                    s->fatal = HASF_EDEVICE;
                    snprintf(s->err, sizeof s->err, "serve kernel launch: %s", hipGetErrorString(e));
                } else {
                    s->kernel_running = true;
                    ++s->launches;
                }
            }
        }
        // retire completed frames
        for (size_t k = 0; k < s->inflight.size();) {
            Frame* f = s->inflight[k];
            const int w = __atomic_load_n(s->done + f->slot, __ATOMIC_ACQUIRE);
            if (w == (int)(f->seq & 0x3FFFFFFFull) + 1) {
                f->t_done = now_s();
                f->done = true;
                s->pool.release(f->off / 256, f->lay.total() / 256);
                s->slot_frame[f->slot] = nullptr;
                s->inflight[k] = s->inflight.back();
                s->inflight.pop_back();
                ++s->completed;
                s->t_last = f->t_done;
                s->px_done += (double)f->img.H * f->img.W;
                s->lat_ms.push_back((f->t_done - f->t_submit) * 1e3);
                progress = true;
            } else {
                ++k;
            }
        }
        if (s->fatal != HASF_OK) {
            // fail everything still queued
            for (Frame* f : s->pending) {
                f->status = s->fatal;
                f->done = true;
            }
            s->pending.clear();
            if (!s->inflight.empty() && !s->kernel_running) {
                for (Frame* f : s->inflight) {
                    f->status = s->fatal;
                    f->done = true;
                    s->slot_frame[f->slot] = nullptr;
                }
                s->inflight.clear();
            }
        }
        if (progress)
            s->cv_done.notify_all();
        if (s->stopping && s->pending.empty() && s->inflight.empty())
            break;
        if (s->pending.empty() && s->inflight.empty()) {
            s->cv_work.wait(lk);
        } else {
            // frames on the device: poll their completion words
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(progress ? 5 : 20));
            lk.lock();
        }
    }
}

hasf_status serve_err(const char* msg)
{
    (void)msg;
    return HASF_EINVAL;
}

}  // namespace

extern "C" {

hasf_status hasf_serve(hasf_ctx* ctx, const hasf_serve_opts* opts, hasf_server** out)
{
    if (!ctx || !out)
        return serve_err("hasf_serve: ctx and out must not be NULL");
    *out = nullptr;
    hasf_serve_opts o{};
    if (opts)
        o = *opts;
    if (o.flags != 0 || o.ring_slots < 0 || o.max_pending < 0 || o.idle_exit_ms < 0)
        return HASF_EINVAL;
    hasf_server* s = new (std::nothrow) hasf_server();
    if (!s)
        return HASF_ENOMEM;
    s->ctx = ctx;
    s->cap = o.ring_slots ? o.ring_slots : 4096;
    s->max_pending = o.max_pending ? o.max_pending : (1 << 20);
    const double idle_ms = o.idle_exit_ms ? o.idle_exit_ms : 2000;
    s->idle_ticks = (unsigned long long)(idle_ms * 1e5);  // 100 MHz wall clock
    const size_t pool_bytes = (o.pool_bytes ? o.pool_bytes : ctx->hbm_budget) / 256 * 256;
    s->lds_cap = std::min(ctx->lds_per_block, (size_t)160 * 1024) - 2048;
    hipSetDevice(ctx->device);
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    const unsigned hflags = hipHostMallocMapped | hipHostMallocCoherent;
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&s->ring, sizeof(ImgDesc) * s->cap, hflags);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&s->tail, 256, hflags);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&s->done, sizeof(int) * s->cap, hflags);
    if (e == hipSuccess) {
        s->stop = (int*)(s->tail + 8);
        *s->tail = 0;
        *s->stop = 0;
        std::memset(s->done, 0, sizeof(int) * s->cap);
        e = hipHostGetDevicePointer((void**)&s->d_ring, s->ring, 0);
    }
    if (e == hipSuccess)
        e = hipHostGetDevicePointer((void**)&s->d_tail, s->tail, 0);
    if (e == hipSuccess)
        e = hipHostGetDevicePointer((void**)&s->d_done, s->done, 0);
    if (e == hipSuccess) {
        s->d_stop = (int*)(s->d_tail + 8);
        e = hipMalloc((void**)&s->head, 256);
    }
    if (e == hipSuccess)
        e = hipMemset(s->head, 0, 256);
    if (e == hipSuccess)
        e = hipMalloc((void**)&s->dev_desc, sizeof(ImgDesc) * s->cap);
    if (e == hipSuccess)
        e = hipMalloc((void**)&s->pool_mem, pool_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        hasf_status st = e == hipErrorOutOfMemory ? HASF_ENOMEM : HASF_EDEVICE;
        if (s->pool_mem) hipFree(s->pool_mem);
        if (s->dev_desc) hipFree(s->dev_desc);
        if (s->head) hipFree(s->head);
        if (s->done) hipHostFree(s->done);
        if (s->tail) hipHostFree(s->tail);
        if (s->ring) hipHostFree(s->ring);
        if (s->stream) hipStreamDestroy(s->stream);
        delete s;
        return st;
    }
    s->pool.init(pool_bytes / 256);
    s->slot_frame.assign(s->cap, nullptr);
    // LDS for any frame that fits; two workgroups per CU
    s->lds_launch = s->lds_cap;
    {
        // the largest LDS image state under the cap
        s->lds_launch = std::min(s->lds_cap, (size_t)78 * 1024);
    }
    s->grid = ctx->num_cu * std::max(1, serve_occupancy(s->lds_launch));
    s->worker = std::thread(serve_loop, s);
    *out = s;
    return HASF_OK;
}

hasf_status hasf_serve_submit(hasf_server* s, const hasf_image* img, uint64_t* ticket)
{
    if (!s || !img || !ticket)
        return HASF_EINVAL;
    if (!img->X || img->H < 1 || img->W < 1 || (int64_t)img->H + img->W > 65535 || img->ld < img->W ||
        img->r < 0 || img->r > HASF_R_MAX) {
        std::lock_guard<std::mutex> g(s->mu);
        ++s->rejected;
        return HASF_EINVAL;
    }
    Frame* f = new (std::nothrow) Frame();
    if (!f)
        return HASF_ENOMEM;
    f->img = *img;
    f->lay = image_layout(img->H, img->W, img->r, s->lds_cap);
    if (f->lay.lds && f->lay.lds_bytes > s->lds_launch) {
        // state fits in LDS but not in what the server kernel was launched with
        f->lay = image_layout(img->H, img->W, img->r, 0);
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stopping || s->fatal != HASF_OK) {
            delete f;
            return s->fatal != HASF_OK ? (hasf_status)s->fatal : HASF_EINVAL;
        }
        if (f->lay.total() > s->pool.size * 256) {
            ++s->rejected;
            delete f;
            return HASF_ENOMEM;  // can never be admitted
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
    out->in_flight = s->inflight.size();
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
    __atomic_store_n(s->stop, 1, __ATOMIC_RELEASE);
    hipSetDevice(s->ctx->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    const int fatal = s->fatal;
    for (auto& kv : s->frames)
        delete kv.second;
    hipFree(s->pool_mem);
    hipFree(s->dev_desc);
    hipFree(s->head);
    hipHostFree(s->done);
    hipHostFree(s->tail);
    hipHostFree(s->ring);
    hipStreamDestroy(s->stream);
    delete s;
    if (e != hipSuccess)
        return HASF_EDEVICE;
    return fatal == HASF_OK ? HASF_OK : (hasf_status)fatal;
}

}  // extern "C"
