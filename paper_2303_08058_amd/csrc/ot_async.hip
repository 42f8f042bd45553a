// ot_async.hip -- host futures for asynchronous launches, completed by event
// polling from the threads that do other work (paper Sec. 3: futures are
// made ready from GPU events by a poll function that the task scheduler
// calls between tasks; one thread polls at a time, others skip; events not
// yet complete are kept and queried again at the next poll).
//
// HIP form of that design:
//  * an executor owns a pool of HIP streams (default priority, created on
//    first use) and a task queue served by optional worker threads;
//  * a future for the work enqueued so far on a stream is an event recorded
//    on it (hipEventDisableTiming, recycled through a free list) plus a
//    reference-counted shared state; registering it is a lock-free push onto
//    a multi-producer stack, so launching threads never block;
//  * poll: try-lock (a thread finding the poller busy returns at once),
//    drain the stack, hipEventQuery every pending event, complete the ready
//    ones and keep the rest for the next poll. No call ever blocks on the
//    GPU (no hipEventSynchronize / hipStreamSynchronize);
//  * continuations of a completed future are posted to the task queue and
//    run by a worker (or, without workers, by whichever thread polls or
//    waits), never while the poll lock is held;
//  * workers run tasks and poll between them while events are pending.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <utility>
#include <vector>

#include "ot_common.h"
#include "ot_fmm.h"

using namespace otfmm;

namespace {

struct Task {
    ot_fmm_callback fn;
    void* user;
};

struct Pending {
    hipEvent_t ev;
    ot_fmm_future_s* fut;
    Pending* next;
};

}  // namespace

struct ot_fmm_future_s {
    std::atomic<int> refs{1};
    std::atomic<bool> ready{false};
    int status = OT_FMM_OK;  // written before `ready` is released
    bool host = false;       // made ready by ot_fmm_future_set_ready, not by an event
    std::mutex mu;
    std::vector<Task> conts;
    ot_fmm_executor_s* ex = nullptr;
};

struct ot_fmm_executor_s {
    std::atomic<int> device{-1};  // fixed by the first GPU use
    int nstreams = 0;
    std::mutex stream_mu;
    std::vector<hipStream_t> streams;
    std::atomic<unsigned> next_stream{0};

    std::atomic<Pending*> incoming{nullptr};  // lock-free registration stack
    std::atomic<long> outstanding{0};         // registered, not yet completed
    std::mutex poll_mu;                       // held by the one polling thread
    std::vector<Pending*> retry;              // owned by the poller

    std::mutex ev_mu;
    std::vector<hipEvent_t> free_events;

    std::mutex task_mu;
    std::condition_variable task_cv;
    std::deque<Task> tasks;
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace {

void future_unref(ot_fmm_future_s* f)
{
    if (f->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) delete f;
}

void post_task(ot_fmm_executor_s* ex, Task t)
{
    {
        std::lock_guard<std::mutex> lk(ex->task_mu);
        ex->tasks.push_back(t);
    }
    ex->task_cv.notify_one();
}

bool pop_task(ot_fmm_executor_s* ex, Task* t)
{
    std::lock_guard<std::mutex> lk(ex->task_mu);
    if (ex->tasks.empty()) return false;
    *t = ex->tasks.front();
    ex->tasks.pop_front();
    return true;
}

// Marks the future ready and posts its continuations (called without the
// poll lock held); false if it was ready already (nothing changes then).
bool complete(ot_fmm_future_s* f, int status)
{
    std::vector<Task> conts;
    {
        std::lock_guard<std::mutex> lk(f->mu);
        if (f->ready.load(std::memory_order_relaxed)) return false;
        f->status = status;
        f->ready.store(true, std::memory_order_release);
        conts.swap(f->conts);
    }
    for (const Task& t : conts) post_task(f->ex, t);
    return true;
}

int get_event(ot_fmm_executor_s* ex, hipEvent_t* ev)
{
    {
        std::lock_guard<std::mutex> lk(ex->ev_mu);
        if (!ex->free_events.empty()) {
            *ev = ex->free_events.back();
            ex->free_events.pop_back();
            return OT_FMM_OK;
        }
    }
    hipError_t e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    return e == hipSuccess ? OT_FMM_OK : hip_fail(e, "hipEventCreateWithFlags");
}

void put_event(ot_fmm_executor_s* ex, hipEvent_t ev)
{
    std::lock_guard<std::mutex> lk(ex->ev_mu);
    ex->free_events.push_back(ev);
}

// One poll; returns the number of futures completed, or -1 when another
// thread is polling.
int poll_once(ot_fmm_executor_s* ex)
{
    std::vector<std::pair<ot_fmm_future_s*, int>> done;
    {
        std::unique_lock<std::mutex> lk(ex->poll_mu, std::try_to_lock);
        if (!lk.owns_lock()) return -1;
        Pending* head = ex->incoming.exchange(nullptr, std::memory_order_acq_rel);
        const size_t first = ex->retry.size();
        for (Pending* p = head; p; p = p->next) ex->retry.push_back(p);
        std::reverse(ex->retry.begin() + first, ex->retry.end());  // registration order
        size_t keep = 0;
        for (size_t i = 0; i < ex->retry.size(); ++i) {
            Pending* p = ex->retry[i];
            const hipError_t e = hipEventQuery(p->ev);
            if (e == hipErrorNotReady) {
                ex->retry[keep++] = p;
                continue;
            }
            int st = OT_FMM_OK;
            if (e != hipSuccess) st = hip_fail(e, "hipEventQuery");
            put_event(ex, p->ev);
            done.emplace_back(p->fut, st);
            delete p;
        }
        ex->retry.resize(keep);
    }
    for (auto& d : done) {
        (void)complete(d.first, d.second);
        future_unref(d.first);  // the registration's reference
        ex->outstanding.fetch_sub(1, std::memory_order_acq_rel);
    }
    return (int)done.size();
}

void worker_loop(ot_fmm_executor_s* ex)
{
    int idle = 0;
    for (;;) {
        Task t;
        if (pop_task(ex, &t)) {
            t.fn(t.user);
            idle = 0;
            continue;
        }
        if (ex->outstanding.load(std::memory_order_acquire) > 0) {
            if (poll_once(ex) > 0) {
                idle = 0;
            } else if (++idle > 64) {
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            } else {
                std::this_thread::yield();
            }
            continue;
        }
        std::unique_lock<std::mutex> lk(ex->task_mu);
        if (ex->stop && ex->tasks.empty()) return;
        ex->task_cv.wait_for(lk, std::chrono::milliseconds(2), [ex] {
            return ex->stop || !ex->tasks.empty() ||
                   ex->outstanding.load(std::memory_order_acquire) > 0;
        });
    }
}

// Stream i of the pool, created on first use on the current device.
int pool_stream(ot_fmm_executor_s* ex, int i, hipStream_t* s)
{
    std::lock_guard<std::mutex> lk(ex->stream_mu);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (ex->device < 0) {
        int rc = ensure_device();
        if (rc) return rc;
        ex->device = dev;
    } else if (dev != ex->device) {
        return fail(OT_FMM_EINVAL, "executor belongs to another device");
    }
    if (!ex->streams[i]) {
        e = hipStreamCreateWithFlags(&ex->streams[i], hipStreamNonBlocking);
        if (e != hipSuccess) {
            ex->streams[i] = nullptr;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
    }
    *s = ex->streams[i];
    return OT_FMM_OK;
}

int register_event(ot_fmm_executor_s* ex, hipStream_t stream, ot_fmm_future* out)
{
    hipEvent_t ev;
    int rc = get_event(ex, &ev);
    if (rc) return rc;
    hipError_t e = hipEventRecord(ev, stream);
    if (e != hipSuccess) {
        put_event(ex, ev);
        return hip_fail(e, "hipEventRecord");
    }
    auto* f = new (std::nothrow) ot_fmm_future_s();
    auto* p = new (std::nothrow) Pending();
    if (!f || !p) {
        delete f;
        delete p;
        (void)hipEventSynchronize(ev);  // recorded: let it finish before reuse
        put_event(ex, ev);
        return fail(OT_FMM_ENOMEM, "host allocation failed");
    }
    f->ex = ex;
    f->refs.store(2, std::memory_order_relaxed);  // caller + registration
    p->ev = ev;
    p->fut = f;
    ex->outstanding.fetch_add(1, std::memory_order_acq_rel);
    Pending* head = ex->incoming.load(std::memory_order_relaxed);
    do {
        p->next = head;
    } while (!ex->incoming.compare_exchange_weak(head, p, std::memory_order_release,
                                                 std::memory_order_relaxed));
    ex->task_cv.notify_one();
    *out = f;
    return OT_FMM_OK;
}

// Runs queued tasks on the calling thread (executors without workers).
void drain_tasks(ot_fmm_executor_s* ex)
{
    Task t;
    while (pop_task(ex, &t)) t.fn(t.user);
}

}  // namespace

extern "C" {

int ot_fmm_executor_create(int nstreams, int nworkers, ot_fmm_executor* out)
{
    g_last_error.clear();
    if (!out) return fail(OT_FMM_EINVAL, "null output pointer");
    *out = nullptr;
    if (nstreams < 1 || nstreams > 1024 || nworkers < 0 || nworkers > 256)
        return fail(OT_FMM_EINVAL, "need 1 <= nstreams <= 1024 and 0 <= nworkers <= 256");
    auto* ex = new (std::nothrow) ot_fmm_executor_s();
    if (!ex) return fail(OT_FMM_ENOMEM, "host allocation failed");
    ex->nstreams = nstreams;
    ex->streams.assign(nstreams, nullptr);
    try {
        for (int i = 0; i < nworkers; ++i) ex->workers.emplace_back(worker_loop, ex);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(ex->task_mu);
            ex->stop = true;
        }
        ex->task_cv.notify_all();
        for (auto& w : ex->workers) w.join();
        delete ex;
        return fail(OT_FMM_ENOMEM, "cannot start worker threads");
    }
    *out = ex;
    return OT_FMM_OK;
}

int ot_fmm_executor_destroy(ot_fmm_executor ex)
{
    g_last_error.clear();
    if (!ex) return OT_FMM_OK;
    // every registered event completes (polling, no blocking wait), then the
    // remaining tasks run and the workers stop
    while (ex->outstanding.load(std::memory_order_acquire) > 0) {
        if (poll_once(ex) <= 0) std::this_thread::yield();
        if (ex->workers.empty()) drain_tasks(ex);
    }
    {
        std::lock_guard<std::mutex> lk(ex->task_mu);
        ex->stop = true;
    }
    ex->task_cv.notify_all();
    for (auto& w : ex->workers) w.join();
    drain_tasks(ex);
    for (hipEvent_t e : ex->free_events) (void)hipEventDestroy(e);
    for (hipStream_t s : ex->streams)
        if (s) (void)hipStreamDestroy(s);
    delete ex;
    return OT_FMM_OK;
}

int ot_fmm_executor_stream(ot_fmm_executor ex, int i, void** stream)
{
    g_last_error.clear();
    if (!ex || !stream || i < 0 || i >= ex->nstreams) return fail(OT_FMM_EINVAL, "bad executor stream query");
    hipStream_t s = nullptr;
    int rc = pool_stream(ex, i, &s);
    if (rc) return rc;
    *stream = (void*)s;
    return OT_FMM_OK;
}

int ot_fmm_executor_get_future(ot_fmm_executor ex, void* stream, ot_fmm_future* out)
{
    g_last_error.clear();
    if (!ex || !out) return fail(OT_FMM_EINVAL, "null executor or output pointer");
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int have = ex->device.load(std::memory_order_acquire);
    if (have >= 0 && dev != have) return fail(OT_FMM_EINVAL, "executor belongs to another device");
    if (have < 0) {
        int rc = ensure_device();
        if (rc) return rc;
        std::lock_guard<std::mutex> lk(ex->stream_mu);
        have = ex->device.load(std::memory_order_acquire);
        if (have < 0) ex->device.store(dev, std::memory_order_release);
        else if (have != dev) return fail(OT_FMM_EINVAL, "executor belongs to another device");
    }
    return register_event(ex, (hipStream_t)stream, out);
}

int ot_fmm_executor_multipole_async(ot_fmm_executor ex, const double* M, const double* com,
                                    double* L, ot_fmm_future* out)
{
    g_last_error.clear();
    if (!ex || !out) return fail(OT_FMM_EINVAL, "null executor or output pointer");
    *out = nullptr;
    if (!aligned8(M) || !aligned8(com) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int i = (int)(ex->next_stream.fetch_add(1, std::memory_order_relaxed) % ex->nstreams);
    hipStream_t s = nullptr;
    int rc = pool_stream(ex, i, &s);
    if (rc) return rc;
    rc = ot_fmm_multipole(M, com, L, (void*)s);
    if (rc) return rc;
    return register_event(ex, s, out);
}

int ot_fmm_executor_post(ot_fmm_executor ex, ot_fmm_callback fn, void* user)
{
    g_last_error.clear();
    if (!ex || !fn) return fail(OT_FMM_EINVAL, "null executor or callback");
    post_task(ex, Task{fn, user});
    return OT_FMM_OK;
}

int ot_fmm_executor_poll(ot_fmm_executor ex, int* completed)
{
    g_last_error.clear();
    if (!ex) return fail(OT_FMM_EINVAL, "null executor");
    const int n = poll_once(ex);
    if (ex->workers.empty()) drain_tasks(ex);
    if (completed) *completed = n;
    return OT_FMM_OK;
}

int ot_fmm_executor_outstanding(ot_fmm_executor ex, int64_t* n)
{
    g_last_error.clear();
    if (!ex || !n) return fail(OT_FMM_EINVAL, "null argument");
    *n = ex->outstanding.load(std::memory_order_acquire);
    return OT_FMM_OK;
}

int ot_fmm_future_create(ot_fmm_executor ex, ot_fmm_future* out)
{
    g_last_error.clear();
    if (!ex || !out) return fail(OT_FMM_EINVAL, "null executor or output pointer");
    auto* f = new (std::nothrow) ot_fmm_future_s();
    if (!f) return fail(OT_FMM_ENOMEM, "host allocation failed");
    f->ex = ex;
    f->host = true;
    *out = f;
    return OT_FMM_OK;
}

int ot_fmm_future_set_ready(ot_fmm_future f)
{
    g_last_error.clear();
    if (!f) return fail(OT_FMM_EINVAL, "null future");
    if (!f->host) return fail(OT_FMM_EINVAL, "future is completed by its GPU event");
    if (!complete(f, OT_FMM_OK)) return fail(OT_FMM_EINVAL, "future already ready");
    return OT_FMM_OK;
}

int ot_fmm_future_then(ot_fmm_future f, ot_fmm_callback fn, void* user)
{
    g_last_error.clear();
    if (!f || !fn) return fail(OT_FMM_EINVAL, "null future or callback");
    {
        std::lock_guard<std::mutex> lk(f->mu);
        if (!f->ready.load(std::memory_order_acquire)) {
            f->conts.push_back(Task{fn, user});
            return OT_FMM_OK;
        }
    }
    post_task(f->ex, Task{fn, user});
    return OT_FMM_OK;
}

int ot_fmm_future_is_ready(ot_fmm_future f, int* ready)
{
    g_last_error.clear();
    if (!f || !ready) return fail(OT_FMM_EINVAL, "null argument");
    *ready = f->ready.load(std::memory_order_acquire) ? 1 : 0;
    return OT_FMM_OK;
}

int ot_fmm_future_wait(ot_fmm_future f, double timeout_s)
{
    g_last_error.clear();
    if (!f) return fail(OT_FMM_EINVAL, "null future");
    ot_fmm_executor_s* ex = f->ex;
    const auto t0 = std::chrono::steady_clock::now();
    int idle = 0;
    while (!f->ready.load(std::memory_order_acquire)) {
        Task t;
        if (pop_task(ex, &t)) {  // help: run a queued task while waiting
            t.fn(t.user);
            continue;
        }
        if (poll_once(ex) <= 0) {
            if (++idle > 64)
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            else
                std::this_thread::yield();
        }
        if (timeout_s >= 0.0 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > timeout_s)
            return fail(OT_FMM_ETIMEDOUT, "future not ready within the time limit");
    }
    if (ex->workers.empty()) drain_tasks(ex);
    if (f->status != OT_FMM_OK) return fail(f->status, "the GPU work behind this future failed");
    return OT_FMM_OK;
}

int ot_fmm_future_release(ot_fmm_future f)
{
    g_last_error.clear();
    if (f) future_unref(f);
    return OT_FMM_OK;
}

}  // extern "C"
