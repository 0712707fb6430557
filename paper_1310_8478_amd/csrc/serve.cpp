// Continuous-batching job server of libdpsnn: admission by device footprint,
// network generation on a build stream, and one batched step over every
// running job, with jobs joining and leaving between quanta.  All device work
// runs in the kernels of build.hip and step.hip; this file only sequences it.
//
// Threads and ownership:
//   builder  pops the head of the submission queue when its footprint fits
//            the budget, generates its network on s_build (the build call
//            returns once the generation has completed), and hands it to the
//            stepper through `ready`;
//   stepper  owns the running jobs and the launch tables of their groups; it
//            launches a quantum on s_step, records an event, and then waits
//            for the previous quantum's event, so the host runs at most one
//            quantum ahead.  Jobs whose last step is in a quantum become DONE
//            when that quantum's event has completed; tables replaced before
//            a quantum are freed when that quantum has completed.
// Every field shared between threads is guarded by `mu`; a job's network is
// touched only by the thread that holds the job (builder, then stepper, then
// the client once the job is DONE).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "net.h"

using namespace dpsnn;

namespace {

struct Job {
    uint64_t id = 0;
    dpsnn_config cfg;
    uint32_t steps = 0;
    uint64_t footprint = 0;
    bool reserved = false;        // footprint counted in the budget
    int status = DPSNN_JOB_QUEUED;
    int error = 0;
    std::string message;
    Net* net = nullptr;
    bool cancel = false;          // dpsnn_server_cancel asked for it (guarded by mu)
    uint32_t launched = 0;
    double t_submit = 0, t_admit = 0, t_built = 0, t_done = 0;
};

// Jobs stepped with one launch per kernel, and the tables of that launch.
struct Group {
    std::vector<Job*> jobs;
    std::vector<Net*> members;
    LaunchSet L;
    std::vector<Net::Alloc> allocs;
};

// A quantum in flight: its completion event, the jobs whose last step it
// holds (or that a failed launch stopped), and tables that became free to
// release once it completes.
struct Quantum {
    hipEvent_t ev = nullptr;
    std::vector<Job*> finishing;
    std::vector<std::unique_ptr<Group>> retired;
};

// Stream-ordered allocation for servers created without callbacks.
void* ordered_alloc(size_t bytes, void* stream, void*) {
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, (hipStream_t)stream) != hipSuccess) return nullptr;
    return p;
}

void ordered_free(void* p, size_t, void* stream, void*) {
    if (p) (void)hipFreeAsync(p, (hipStream_t)stream);
}

}  // namespace

struct dpsnn_server {
    dpsnn_device dev{};           // device and allocator of every job
    bool own_pool = false;        // allocations come from the device's default pool
    hipStream_t s_build = nullptr, s_step = nullptr, s_read = nullptr;
    std::chrono::steady_clock::time_point t0;
    uint64_t budget = 0, reserved = 0, peak_reserved = 0;
    uint32_t max_quantum = 8, max_jobs = 256;
    Tuning tune;
    Timers timers;                // stays off: quanta are not bracketed

    std::mutex mu;
    std::condition_variable cv_admit, cv_ready, cv_done;
    std::deque<Job*> queue;       // QUEUED, in submission order
    std::deque<Job*> ready;       // built, not yet stepping
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    std::deque<uint64_t> finished;  // DONE or FAILED, not yet returned by wait_any
    uint64_t next_id = 1;
    uint32_t admitted = 0;        // RUNNING jobs
    bool stop = false;
    dpsnn_server_stats st{};
    std::thread builder, stepper;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void builder_main();
    void stepper_main();
    int make_groups(const std::vector<Job*>& active, std::vector<std::unique_ptr<Group>>& out);
    void complete(Quantum& q, std::vector<hipEvent_t>& pool);
    // with mu held: the job leaves the running set
    void finish_locked(Job* j, double t, int error, const std::string& msg);
};

void dpsnn_server::finish_locked(Job* j, double t, int error, const std::string& msg) {
    if (j->status == DPSNN_JOB_RUNNING && admitted) admitted--;
    j->status = error ? DPSNN_JOB_FAILED : DPSNN_JOB_DONE;
    j->error = error;
    j->message = msg;
    j->t_done = t;
    if (j->net) {
        j->net->in_batch = false;
        j->net->stream = s_read;
    }
    if (error) st.failed++;
    else st.completed++;
    finished.push_back(j->id);
}

void dpsnn_server::builder_main() {
    (void)hipSetDevice(dev.device);
    dpsnn_device bdev = dev;
    bdev.stream = s_build;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_admit.wait(lk, [&] {
            return stop || (!queue.empty() && admitted < max_jobs &&
                            reserved + queue.front()->footprint <= budget);
        });
        if (stop) return;
        Job* j = queue.front();
        queue.pop_front();
        j->status = DPSNN_JOB_RUNNING;
        j->t_admit = now();
        j->reserved = true;
        reserved += j->footprint;
        peak_reserved = std::max(peak_reserved, reserved);
        admitted++;
        st.peak_running = std::max<uint64_t>(st.peak_running, admitted);
        const dpsnn_config cfg = j->cfg;
        lk.unlock();

        dpsnn_net* h = nullptr;
        const int rc = dpsnn_build_network(&cfg, &bdev, &h);
        const std::string msg = rc ? std::string(dpsnn_last_error()) : std::string();
        Net* n = reinterpret_cast<Net*>(h);
        if (n) {
            n->owner = this;
            n->in_batch = true;
        }

        lk.lock();
        if (rc) {
            j->reserved = false;
            reserved -= j->footprint;
            finish_locked(j, now(), rc, msg);
            cv_done.notify_all();
            continue;
        }
        j->net = n;
        if (j->cancel) {  // cancelled while it was being built: never stepped
            j->t_built = now();
            finish_locked(j, j->t_built, DPSNN_E_CANCELED, "cancelled");
            cv_done.notify_all();
            continue;
        }
        j->t_built = now();
        ready.push_back(j);
        cv_ready.notify_one();
    }
}

int dpsnn_server::make_groups(const std::vector<Job*>& active,
                              std::vector<std::unique_ptr<Group>>& out) {
    for (Job* j : active) {
        Net* n = j->net;
        Group* g = nullptr;
        if (n->cfg.sum_mode != DPSNN_SUM_ORDERED) {
            for (auto& x : out) {
                const Net* m = x->members[0];
                if (m->cfg.sum_mode == n->cfg.sum_mode && m->tgt16 == n->tgt16) {
                    g = x.get();
                    break;
                }
            }
        }
        if (!g) {
            out.push_back(std::make_unique<Group>());
            g = out.back().get();
        }
        g->jobs.push_back(j);
        g->members.push_back(n);
    }
    dpsnn_device sdev = dev;
    sdev.stream = s_step;
    for (auto& g : out) {
        const int rc = make_launch_set(g->L, g->members.data(), (uint32_t)g->members.size(), sdev,
                                       s_step, &g->allocs, false);
        if (rc) return rc;
    }
    return DPSNN_OK;
}

void dpsnn_server::complete(Quantum& q, std::vector<hipEvent_t>& pool) {
    hipError_t e = q.ev ? hipEventSynchronize(q.ev) : hipStreamSynchronize(s_step);
    const double t = now();
    {
        std::lock_guard<std::mutex> lk(mu);
        for (Job* j : q.finishing) {
            if (j->error == 0 && e != hipSuccess)
                j->error = DPSNN_E_DEVICE, j->message = hipGetErrorString(e);
            finish_locked(j, t, j->error, j->message);
        }
    }
    if (!q.finishing.empty()) {
        cv_done.notify_all();
        cv_admit.notify_one();
    }
    dpsnn_device sdev = dev;
    for (auto& g : q.retired) {
        release_launch_set_host(g->L);
        free_tracked(sdev, s_step, g->allocs);
    }
    q.retired.clear();
    if (q.ev) pool.push_back(q.ev);
    q.ev = nullptr;
}

void dpsnn_server::stepper_main() {
    (void)hipSetDevice(dev.device);
    std::vector<Job*> active;
    std::vector<std::unique_ptr<Group>> groups;
    std::deque<Quantum> inflight;
    std::vector<hipEvent_t> pool;
    bool regroup = false;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            if (active.empty() && inflight.empty())
                cv_ready.wait(lk, [&] { return stop || !ready.empty(); });
            if (stop) break;
            bool dropped = false;
            while (!ready.empty()) {
                Job* j = ready.front();
                ready.pop_front();
                if (j->cancel) {  // built but never stepped
                    finish_locked(j, now(), DPSNN_E_CANCELED, "cancelled");
                    dropped = true;
                    continue;
                }
                active.push_back(j);
                regroup = true;
            }
            if (dropped) cv_done.notify_all();
        }
        if (active.empty()) {  // nothing to launch: retire what is in flight
            complete(inflight.front(), pool);
            inflight.pop_front();
            continue;
        }
        Quantum qm;
        int err = DPSNN_OK;
        std::string msg;
        if (regroup) {
            for (auto& g : groups) qm.retired.push_back(std::move(g));
            groups.clear();
            err = make_groups(active, groups);
            if (err) {
                msg = "launch tables: " + std::string(dpsnn_last_error());
                for (auto& g : groups) qm.retired.push_back(std::move(g));
                groups.clear();
            }
            regroup = false;
        }
        uint32_t q = max_quantum;
        for (Job* j : active) q = std::min(q, j->steps - j->net->t);
        hipError_t e = hipSuccess;
        for (uint32_t s = 0; s < q && !err && e == hipSuccess; ++s)
            for (auto& g : groups) {
                e = launch_step_set(g->L, tune, timers, s_step, g->members.data());
                if (e != hipSuccess) break;
            }
        if (!err && e != hipSuccess) {
            err = DPSNN_E_DEVICE;
            msg = std::string("step launch: ") + hipGetErrorString(e);
        }
        if (!pool.empty()) {
            qm.ev = pool.back();
            pool.pop_back();
        } else if (hipEventCreateWithFlags(&qm.ev, hipEventDisableTiming) != hipSuccess) {
            qm.ev = nullptr;
        }
        if (qm.ev && hipEventRecord(qm.ev, s_step) != hipSuccess) {
            (void)hipEventDestroy(qm.ev);
            qm.ev = nullptr;
        }
        std::vector<Job*> keep;
        {
            std::lock_guard<std::mutex> lk(mu);
            st.quanta++;
            if (!err) st.set_steps += (uint64_t)q * groups.size();
            for (Job* j : active) {
                st.job_steps += j->net->t - j->launched;
                j->launched = j->net->t;
            }
            // a job leaves after this quantum when it failed, finished or was
            // cancelled; its network is touched by no later quantum
            for (Job* j : active) {
                if (err) {
                    j->error = err;
                    j->message = msg;
                    qm.finishing.push_back(j);
                } else if (j->net->t >= j->steps) {
                    qm.finishing.push_back(j);
                } else if (j->cancel) {
                    j->error = DPSNN_E_CANCELED;
                    j->message = "cancelled";
                    qm.finishing.push_back(j);
                } else {
                    keep.push_back(j);
                }
            }
        }
        if (keep.size() != active.size()) regroup = true;
        active.swap(keep);
        if (err) {
            for (auto& g : groups) qm.retired.push_back(std::move(g));
            groups.clear();
        }
        inflight.push_back(std::move(qm));
        while (inflight.size() > 1 || (active.empty() && !inflight.empty())) {
            complete(inflight.front(), pool);
            inflight.pop_front();
        }
    }
    // shutting down: let the launched quanta finish, stop the rest
    while (!inflight.empty()) {
        complete(inflight.front(), pool);
        inflight.pop_front();
    }
    (void)hipStreamSynchronize(s_step);
    {
        std::lock_guard<std::mutex> lk(mu);
        const double t = now();
        for (Job* j : active) finish_locked(j, t, DPSNN_E_INVAL, "server shut down");
    }
    cv_done.notify_all();
    dpsnn_device sdev = dev;
    for (auto& g : groups) {
        release_launch_set_host(g->L);
        free_tracked(sdev, s_step, g->allocs);
    }
    for (hipEvent_t ev : pool) (void)hipEventDestroy(ev);
}

namespace {

void fill_info(const Job& j, dpsnn_job_info* info) {
    std::memset(info, 0, sizeof(*info));
    info->id = j.id;
    info->status = j.status;
    info->error = j.error;
    info->steps = j.steps;
    info->steps_launched = j.launched;
    info->footprint = j.footprint;
    info->t_submit = j.t_submit;
    info->t_admit = j.t_admit;
    info->t_built = j.t_built;
    info->t_done = j.t_done;
    info->net = j.status == DPSNN_JOB_DONE ? reinterpret_cast<dpsnn_net*>(j.net) : nullptr;
    std::strncpy(info->message, j.message.c_str(), sizeof(info->message) - 1);
}

bool is_final(int status) { return status == DPSNN_JOB_DONE || status == DPSNN_JOB_FAILED; }

}  // namespace

extern "C" {

int dpsnn_server_create(const dpsnn_device* dev, uint64_t budget_bytes, uint32_t max_quantum,
                        uint32_t max_jobs, dpsnn_server** out) {
    if (!out) return fail(DPSNN_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!dev) return fail(DPSNN_E_INVAL, "device is NULL");
    if ((dev->alloc == nullptr) != (dev->free == nullptr))
        return fail(DPSNN_E_INVAL, "alloc and free callbacks must be given together");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || dev->device < 0 || dev->device >= ndev)
        return fail(DPSNN_E_INVAL, "no such HIP device");
    if (hipSetDevice(dev->device) != hipSuccess) return fail(DPSNN_E_DEVICE, "hipSetDevice");
    std::unique_ptr<dpsnn_server> s(new dpsnn_server());
    s->dev = *dev;
    s->dev.stream = nullptr;
    if (!dev->alloc) {
        s->dev.alloc = ordered_alloc;
        s->dev.free = ordered_free;
        s->dev.ctx = nullptr;
        s->own_pool = true;
        // keep freed blocks in the pool for the next jobs (trimmed at destroy)
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, dev->device) == hipSuccess && pool) {
            uint64_t keep = ~0ull;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
    }
    if (budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(DPSNN_E_DEVICE, "hipMemGetInfo");
        budget_bytes = (uint64_t)((double)fr * 0.9);
    }
    s->budget = budget_bytes;
    s->max_quantum = max_quantum ? max_quantum : 8u;
    s->max_jobs = max_jobs ? max_jobs : 256u;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev->device) == hipSuccess &&
        lds > 0)
        s->tune.max_lds = (size_t)lds;
    if (hipStreamCreateWithFlags(&s->s_build, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->s_step, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->s_read, hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t x : {s->s_build, s->s_step, s->s_read})
            if (x) (void)hipStreamDestroy(x);
        return fail(DPSNN_E_DEVICE, "stream creation failed");
    }
    s->t0 = std::chrono::steady_clock::now();
    s->st.budget_bytes = s->budget;
    dpsnn_server* p = s.get();
    try {
        p->builder = std::thread([p] { p->builder_main(); });
        p->stepper = std::thread([p] { p->stepper_main(); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(p->mu);
            p->stop = true;
        }
        p->cv_admit.notify_all();
        p->cv_ready.notify_all();
        if (p->builder.joinable()) p->builder.join();
        for (hipStream_t x : {p->s_build, p->s_step, p->s_read}) (void)hipStreamDestroy(x);
        return fail(DPSNN_E_INVAL, "could not start the server threads");
    }
    *out = s.release();
    return DPSNN_OK;
}

int dpsnn_server_submit(dpsnn_server* s, const dpsnn_config* cfg, uint32_t steps, uint64_t* job) {
    if (!s || !cfg || !job) return fail(DPSNN_E_INVAL, "NULL argument");
    if (steps < 1 || steps >= (1u << 20)) return fail(DPSNN_E_INVAL, "steps must be in 1 .. 2^20 - 1");
    dpsnn_config c = *cfg;
    if (c.raster_steps == 0) c.raster_steps = std::max(steps + 1u, c.max_delay + 1u);
    uint64_t fp = 0;
    int rc = dpsnn_footprint_bytes(&c, &fp);
    if (rc) return rc;
    if (fp > s->budget) return fail(DPSNN_E_NOMEM, "the job's footprint exceeds the server budget");
    auto j = std::make_unique<Job>();
    j->cfg = c;
    j->steps = steps;
    j->footprint = fp;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(DPSNN_E_INVAL, "the server is shutting down");
        j->id = s->next_id++;
        j->t_submit = s->now();
        *job = j->id;
        s->queue.push_back(j.get());
        s->jobs.emplace(j->id, std::move(j));
        s->st.submitted++;
    }
    s->cv_admit.notify_one();
    return DPSNN_OK;
}

int dpsnn_server_query(dpsnn_server* s, uint64_t job, dpsnn_job_info* info) {
    if (!s || !info) return fail(DPSNN_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(DPSNN_E_INVAL, "unknown or released job");
    fill_info(*it->second, info);
    return DPSNN_OK;
}

int dpsnn_server_wait(dpsnn_server* s, uint64_t job, double timeout_s, dpsnn_job_info* info) {
    if (!s || !info) return fail(DPSNN_E_INVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto gone_or_final = [&] {
        auto it = s->jobs.find(job);
        return s->stop || it == s->jobs.end() || is_final(it->second->status);
    };
    if (s->jobs.find(job) == s->jobs.end()) return fail(DPSNN_E_INVAL, "unknown or released job");
    bool ok = true;
    if (timeout_s < 0) s->cv_done.wait(lk, gone_or_final);
    else ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), gone_or_final);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(DPSNN_E_INVAL, "the job was released while waiting");
    fill_info(*it->second, info);
    if (!ok || !is_final(it->second->status)) return fail(DPSNN_E_TIMEOUT, "the job has not finished");
    // collected here: dpsnn_server_wait_any will not return it again
    auto f = std::find(s->finished.begin(), s->finished.end(), job);
    if (f != s->finished.end()) s->finished.erase(f);
    return DPSNN_OK;
}

int dpsnn_server_cancel(dpsnn_server* s, uint64_t job) {
    if (!s) return fail(DPSNN_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(DPSNN_E_INVAL, "unknown or released job");
    Job* j = it->second.get();
    if (is_final(j->status)) return fail(DPSNN_E_INVAL, "the job has already finished");
    j->cancel = true;
    if (j->status == DPSNN_JOB_QUEUED) {
        auto q = std::find(s->queue.begin(), s->queue.end(), j);
        if (q != s->queue.end()) s->queue.erase(q);
        s->finish_locked(j, s->now(), DPSNN_E_CANCELED, "cancelled");
        s->cv_done.notify_all();
        s->cv_admit.notify_one();  // the next job may now be at the head
    }
    return DPSNN_OK;
}

int dpsnn_server_wait_any(dpsnn_server* s, double timeout_s, dpsnn_job_info* info) {
    if (!s || !info) return fail(DPSNN_E_INVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto have = [&] {
        while (!s->finished.empty() && s->jobs.find(s->finished.front()) == s->jobs.end())
            s->finished.pop_front();
        return s->stop || !s->finished.empty();
    };
    bool ok = true;
    if (timeout_s < 0) s->cv_done.wait(lk, have);
    else ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), have);
    if (!ok || s->finished.empty()) {
        std::memset(info, 0, sizeof(*info));
        return fail(s->stop ? DPSNN_E_INVAL : DPSNN_E_TIMEOUT,
                    s->stop ? "the server is shutting down" : "no job finished in time");
    }
    const uint64_t id = s->finished.front();
    s->finished.pop_front();
    fill_info(*s->jobs.at(id), info);
    return DPSNN_OK;
}

int dpsnn_server_release(dpsnn_server* s, uint64_t job) {
    if (!s) return fail(DPSNN_E_INVAL, "server is NULL");
    std::unique_ptr<Job> j;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(job);
        if (it == s->jobs.end()) return fail(DPSNN_E_INVAL, "unknown or released job");
        if (!is_final(it->second->status)) return fail(DPSNN_E_INVAL, "the job is still queued or running");
        if (it->second->net && it->second->net->in_batch)
            return fail(DPSNN_E_INVAL, "the job's network belongs to a batch");
        j = std::move(it->second);
        s->jobs.erase(it);
    }
    if (j->net) {
        (void)hipSetDevice(s->dev.device);
        j->net->owner = nullptr;
        destroy_net(j->net);
        j->net = nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (j->reserved) s->reserved -= j->footprint;
        s->st.released++;
    }
    s->cv_admit.notify_one();
    return DPSNN_OK;
}

int dpsnn_server_get_stats(dpsnn_server* s, dpsnn_server_stats* out) {
    if (!s || !out) return fail(DPSNN_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = s->queue.size();
    out->running = s->admitted;
    out->budget_bytes = s->budget;
    out->reserved_bytes = s->reserved;
    out->peak_reserved_bytes = s->peak_reserved;
    return DPSNN_OK;
}

int dpsnn_server_clock(dpsnn_server* s, double* seconds) {
    if (!s || !seconds) return fail(DPSNN_E_INVAL, "NULL argument");
    *seconds = s->now();
    return DPSNN_OK;
}

void dpsnn_server_destroy(dpsnn_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_admit.notify_all();
    s->cv_ready.notify_all();
    s->cv_done.notify_all();
    if (s->builder.joinable()) s->builder.join();
    if (s->stepper.joinable()) s->stepper.join();
    (void)hipSetDevice(s->dev.device);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const double t = s->now();
        for (Job* j : s->ready) s->finish_locked(j, t, DPSNN_E_INVAL, "server shut down");
        for (Job* j : s->queue) s->finish_locked(j, t, DPSNN_E_INVAL, "server shut down");
        s->ready.clear();
        s->queue.clear();
    }
    s->cv_done.notify_all();
    for (auto& kv : s->jobs) {
        Job& j = *kv.second;
        if (j.net) {
            j.net->owner = nullptr;
            j.net->in_batch = false;
            destroy_net(j.net);
            j.net = nullptr;
        }
    }
    s->jobs.clear();
    for (hipStream_t x : {s->s_build, s->s_step, s->s_read}) {
        (void)hipStreamSynchronize(x);
        (void)hipStreamDestroy(x);
    }
    if (s->own_pool) {
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, s->dev.device) == hipSuccess && pool)
            (void)hipMemPoolTrimTo(pool, 0);
    }
    s->timers.release();
    delete s;
}

}  // extern "C"
