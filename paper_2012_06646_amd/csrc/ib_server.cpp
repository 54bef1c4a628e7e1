// Serving loop: independent spread/interpolate jobs arrive one by one, wait in a FIFO
// queue, and are admitted into batches by their device-memory footprint within a
// caller-owned arena; each batch runs with one launch per stage (ib_batch_run's path) on
// the server's own stream.  A worker thread forms the batches, launches them and retires
// them in order, recording per-job latency from the (scheduled) arrival to the observed
// completion.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "ib.h"
#include "ib_host.h"
#include "ib_internal.h"
#include "ib_ring.h"

using namespace ibk;

namespace {

constexpr int MAX_INFLIGHT = 4;
constexpr int GRAPH_GRID = 1024;  // blocks per stage in a captured batch graph

struct QueuedJob {
    ib_job job;
    uint64_t ticket;
    double arrival_us;
    size_t bytes;  // plan region
};

struct Result {
    int32_t status;
    double latency_us;
};

struct Flight {
    std::vector<QueuedJob> jobs;
    int slot;
    hipEvent_t done;
};

}  // namespace

struct ib_server_s {
    ib_server_opts opts;
    char* arena;         // slot headers, then the ring of plan regions
    char* plans;         // start of the ring
    size_t header_bytes; // one slot's header (job table for max_jobs_per_batch jobs)
    Ring ring;
    int device;
    hipStream_t stream;
    char* staging;       // pinned: MAX_INFLIGHT slots of slot_bytes
    uint32_t* flags;     // pinned: MAX_INFLIGHT x BATCH_MAX_JOBS
    size_t slot_bytes;
    hipEvent_t events[MAX_INFLIGHT];
    bool slot_busy[MAX_INFLIGHT];
    // With use_graph: one graph per slot and (dimension, kernel), captured on first use; its
    // grids are fixed and its kernels loop over the batch's virtual blocks.
    hipGraphExec_t graphs[MAX_INFLIGHT][2][IB_KERNEL_COUNT];
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<QueuedJob> queue;
    std::deque<Flight> flight;
    std::unordered_map<uint64_t, Result> results;  // finished, not yet reported
    std::unordered_set<uint64_t> open;             // submitted, not yet finished
    uint64_t next_ticket = 1;
    uint64_t pending = 0;  // submitted and not yet finished
    bool stop = false;
    ib_server_stats stats;
    std::thread worker;

    double now_us() const
    {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }

    // Retire the oldest batches whose completion event has fired.  Caller holds mu.
    bool retire()
    {
        bool any = false;
        while (!flight.empty()) {
            Flight& F = flight.front();
            const hipError_t q = hipEventQuery(F.done);
            if (q == hipErrorNotReady) break;
            const double t = now_us();
            const uint32_t* fl = flags + (size_t)F.slot * BATCH_MAX_JOBS;
            for (size_t j = 0; j < F.jobs.size(); ++j) {
                const QueuedJob& J = F.jobs[j];
                const int32_t st = q != hipSuccess ? IB_ERR_HIP : (fl[j] ? IB_ERR_DEVICE_FLAG : IB_OK);
                results[J.ticket] = Result{st, t - J.arrival_us};
                open.erase(J.ticket);
                stats.jobs_done += 1;
                stats.points += (uint64_t)J.job.npts;
            }
            pending -= F.jobs.size();
            slot_busy[F.slot] = false;
            ring.pop();
            flight.pop_front();
            any = true;
        }
        if (any) cv.notify_all();
        return any;
    }

    // Form and launch one batch from the head of the queue.  Caller holds mu.
    bool launch_one()
    {
        if (queue.empty() || (int)flight.size() >= opts.max_inflight) return false;
        int slot = -1;
        for (int s = 0; s < opts.max_inflight; ++s)
            if (!slot_busy[s]) { slot = s; break; }
        if (slot < 0) return false;
        // Admit jobs in arrival order while they share the first job's dimension and kernel
        // and their plan regions still fit in the free part of the arena.
        const ib_job& j0 = queue.front().job;
        size_t body = 0, off = 0;
        int k = 0;
        while (k < (int)queue.size() && k < opts.max_jobs_per_batch) {
            const ib_job& jk = queue[k].job;
            if (jk.grid.dim != j0.grid.dim || jk.grid.kernel != j0.grid.kernel) break;
            size_t o;
            if (!ring.place(body + queue[k].bytes, &o)) break;
            body += queue[k].bytes;
            off = o;
            ++k;
        }
        if (k == 0) return false;  // the arena is busy: wait for a batch to retire
        Flight F;
        F.slot = slot;
        F.done = events[slot];
        std::vector<ib_job> jobs(k);
        for (int i = 0; i < k; ++i) {
            F.jobs.push_back(queue.front());
            jobs[i] = queue.front().job;
            queue.pop_front();
        }
        const size_t total = body;
        char* header = arena + (size_t)slot * header_bytes;
        char* stage = staging + (size_t)slot * slot_bytes;
        uint32_t* fl = flags + (size_t)slot * BATCH_MAX_JOBS;
        BatchLaunch bl;
        int32_t st = batch_prepare(jobs.data(), k, opts.dtype, header, plans + off, total, stage, &bl);
        if (st == IB_OK) {
            if (opts.use_graph < 0 || (opts.use_graph > 0 && k <= opts.use_graph)) {
                st = graph_launch(slot, bl);
            } else {
                const size_t nb = batch_jobs_offset() + (size_t)k * sizeof(BatchJob);
                hipError_t e = hipMemcpyAsync(header, stage, nb, hipMemcpyHostToDevice, stream);
                if (e == hipSuccess) e = launch_batch_plan(bl, stream);
                if (e == hipSuccess) e = launch_batch_ops(bl, stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(fl, header + batch_flags_offset(), k * sizeof(uint32_t),
                                       hipMemcpyDeviceToHost, stream);
                st = hip_status(e);
            }
        }
        if (st == IB_OK && hipEventRecord(F.done, stream) != hipSuccess) st = IB_ERR_HIP;
        if (st != IB_OK) {
            const double t = now_us();
            for (const QueuedJob& J : F.jobs) {
                results[J.ticket] = Result{st, t - J.arrival_us};
                open.erase(J.ticket);
            }
            pending -= k;
            cv.notify_all();
            return true;
        }
        ring.push(off, total);
        slot_busy[slot] = true;
        flight.push_back(std::move(F));
        stats.batches += 1;
        return true;
    }

    // Replay the slot's graph for this batch's dimension and kernel (capturing it first if
    // needed): upload of the whole slot header, every stage with fixed grids, download of
    // the flags.  The header's host copy is already in the slot's staging buffer.
    int32_t graph_launch(int slot, const BatchLaunch& exact)
    {
        const int di = exact.dim == 3 ? 1 : 0, ki = exact.kernel;
        hipGraphExec_t& ge = graphs[slot][di][ki];
        if (!ge) {
            char* header = arena + (size_t)slot * header_bytes;
            BatchLaunch bl = exact;
            for (int s = 0; s < BS_COUNT; ++s) bl.grid[s] = GRAPH_GRID;
            const size_t nb = batch_jobs_offset() + (size_t)opts.max_jobs_per_batch * sizeof(BatchJob);
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return IB_ERR_HIP;
            hipError_t e = hipMemcpyAsync(header, staging + (size_t)slot * slot_bytes, nb,
                                          hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = launch_batch_plan(bl, stream);
            if (e == hipSuccess) e = launch_batch_ops(bl, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(flags + (size_t)slot * BATCH_MAX_JOBS, header + batch_flags_offset(),
                                   BATCH_MAX_JOBS * sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
            const hipError_t e2 = hipStreamEndCapture(stream, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                ge = nullptr;
                return IB_ERR_HIP;
            }
        }
        return hip_status(hipGraphLaunch(ge, stream));
    }

    void run()
    {
        hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            bool progress = retire();
            while (launch_one()) progress = true;
            if (stop && queue.empty() && flight.empty()) break;
            if (progress) continue;
            if (flight.empty()) {
                cv.wait(lk, [&] { return stop || !queue.empty(); });
            } else {
                // Batches in flight: poll their events closely (completion time is latency).
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        }
    }
};

extern "C" {

int32_t ib_server_create(const ib_server_opts* opts, void* arena, size_t arena_bytes, ib_server* out)
{
    if (!opts || !out || !arena || ((uintptr_t)arena % ALIGN) != 0) return IB_ERR_ARG;
    *out = nullptr;
    if (opts->dtype != IB_F64 && opts->dtype != IB_F32) return IB_ERR_UNSUPPORTED;
    if (opts->max_jobs_per_batch < 1 || opts->max_jobs_per_batch > BATCH_MAX_JOBS) return IB_ERR_ARG;
    if (opts->max_inflight < 1 || opts->max_inflight > MAX_INFLIGHT) return IB_ERR_ARG;
    if (opts->max_queue < 1) return IB_ERR_ARG;
    ib_server_s* s = new (std::nothrow) ib_server_s();
    if (!s) return IB_ERR_OOM;
    s->opts = *opts;
    s->arena = (char*)arena;
    s->header_bytes = batch_header_bytes(BATCH_MAX_JOBS);
    const size_t reserved = MAX_INFLIGHT * s->header_bytes;
    if (arena_bytes <= reserved) {
        delete s;
        return IB_ERR_OOM;
    }
    s->plans = s->arena + reserved;
    s->ring.cap = arena_bytes - reserved;
    std::memset(s->graphs, 0, sizeof s->graphs);
    std::memset(&s->stats, 0, sizeof s->stats);
    s->slot_bytes = s->header_bytes;
    bool ok = hipGetDevice(&s->device) == hipSuccess &&
              hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess;
    s->staging = nullptr;
    s->flags = nullptr;
    ok = ok && hipHostMalloc((void**)&s->staging, MAX_INFLIGHT * s->slot_bytes, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->flags, MAX_INFLIGHT * BATCH_MAX_JOBS * sizeof(uint32_t),
                             hipHostMallocDefault) == hipSuccess;
    for (int i = 0; i < MAX_INFLIGHT; ++i) {
        s->slot_busy[i] = false;
        s->events[i] = nullptr;
        ok = ok && hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        for (int i = 0; i < MAX_INFLIGHT; ++i)
            if (s->events[i]) (void)hipEventDestroy(s->events[i]);
        if (s->staging) (void)hipHostFree(s->staging);
        if (s->flags) (void)hipHostFree(s->flags);
        delete s;
        return IB_ERR_HIP;
    }
    s->t0 = std::chrono::steady_clock::now();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return IB_OK;
}

double ib_server_clock_us(ib_server s) { return s ? s->now_us() : -1.0; }

int32_t ib_batch_submit(ib_server s, const ib_job* job, double arrival_us, uint64_t* ticket)
{
    if (!s || !job || !ticket) return IB_ERR_ARG;
    const size_t bytes = batch_job_bytes(job, s->opts.dtype);
    if (bytes == 0) return IB_ERR_ARG;
    if (job->npts > 0 && !job->X) return IB_ERR_ARG;
    if (job->f && job->npts > 0 && !job->F) return IB_ERR_ARG;
    if (job->u && job->npts > 0 && !job->U) return IB_ERR_ARG;
    if (bytes > s->ring.cap) return IB_ERR_OOM;  // can never be admitted
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int64_t)s->queue.size() >= s->opts.max_queue) return IB_ERR_BUSY;
    QueuedJob q;
    q.job = *job;
    q.ticket = s->next_ticket++;
    q.arrival_us = arrival_us >= 0.0 ? arrival_us : s->now_us();
    q.bytes = bytes;
    s->queue.push_back(q);
    s->open.insert(q.ticket);
    s->pending += 1;
    *ticket = q.ticket;
    s->cv.notify_all();
    return IB_OK;
}

int32_t ib_batch_poll(ib_server s, uint64_t ticket, double* latency_us)
{
    if (!s) return IB_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return s->open.count(ticket) ? IB_PENDING : IB_ERR_ARG;
    const Result r = it->second;
    s->results.erase(it);
    if (latency_us) *latency_us = r.latency_us;
    return r.status;
}

int32_t ib_server_drain(ib_server s)
{
    if (!s) return IB_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->pending == 0; });
    return IB_OK;
}

int32_t ib_server_get_stats(ib_server s, ib_server_stats* out)
{
    if (!s || !out) return IB_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return IB_OK;
}

void ib_server_destroy(ib_server s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (int i = 0; i < MAX_INFLIGHT; ++i) {
        (void)hipEventDestroy(s->events[i]);
        for (int d = 0; d < 2; ++d)
            for (int k = 0; k < IB_KERNEL_COUNT; ++k)
                if (s->graphs[i][d][k]) (void)hipGraphExecDestroy(s->graphs[i][d][k]);
    }
    (void)hipStreamDestroy(s->stream);
    (void)hipHostFree(s->staging);
    (void)hipHostFree(s->flags);
    delete s;
}

}  // extern "C"
