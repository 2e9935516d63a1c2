// Serving loop: admits stencil jobs as they arrive (sized by a device arena)
// and keeps their grids resident between sweeps.  Jobs whose plans share
// device tables (one plan class) are swept together, up to 16 grids per
// launch; each class advances on its own stream as soon as its previous
// launch has finished, so classes with short sweeps are not held back by
// classes with long ones, and a job that arrives joins its class's next
// launch.  The worker thread never blocks on the device: it polls events.
#include <hip/hip_runtime.h>

#include <algorithm>
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

#include "../../include/sparstencil.h"
#include "plan.hpp"

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) of the arena, blocks kept sorted.
class Arena {
   public:
    explicit Arena(size_t size) : size_(size) {}
    bool alloc(size_t bytes, size_t *off) {
        bytes = round_up(bytes);
        size_t pos = 0;
        for (auto it = used_.begin(); it != used_.end(); ++it) {
            if (it->first - pos >= bytes) break;
            pos = it->first + it->second;
        }
        if (pos + bytes > size_) return false;
        used_[pos] = bytes;
        *off = pos;
        return true;
    }
    void release(size_t off) { used_.erase(off); }

   private:
    size_t size_;
    std::map<size_t, size_t> used_;  // offset -> bytes
};

// Device work of a job in flight: admission copy, a sweep, or the copy out.
enum Phase { kCopyIn = 0, kSweep = 1, kCopyOut = 2 };

struct Job {
    ss_job_info info{};
    ss_plan_t plan = nullptr;
    const void *in = nullptr;
    void *out = nullptr;
    size_t grid_bytes = 0;
    size_t arena_off = 0;
    char *buf[2] = {nullptr, nullptr};
    int cur = 0;                 // buffer holding the current state
    hipEvent_t done = nullptr;   // completes the job's work in flight
    bool busy = false;           // work in flight
    Phase phase = kCopyIn;
    int advance = 0;             // sweeps the launch in flight applies
};

}  // namespace

struct ss_server_ {
    char *arena_base = nullptr;
    size_t arena_bytes = 0;
    Arena arena;
    int max_jobs = 0;
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> event_pool;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job *> queue;       // submitted, not admitted (FIFO)
    std::vector<Job *> running;    // admitted (worker thread only)
    std::unordered_map<uint64_t, Job *> jobs;
    uint64_t next_id = 1;
    int live = 0;                  // queued + running
    bool stop = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::thread worker;

    explicit ss_server_(size_t bytes) : arena_bytes(bytes), arena(bytes) {}

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    hipEvent_t take_event() {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    // the stream of a plan class (a class's launches stay in order)
    hipStream_t stream_of(const ss_plan_ *p) const { return streams[p->klass % streams.size()]; }
    void run();
    bool step();
    void fail(Job *j, ss_status st) {
        j->info.status = st;
        j->busy = false;
    }
};

// One pass of the worker: retire finished device work, admit queued jobs,
// launch the next sweep of every idle class group.  Returns whether
// anything happened.
bool ss_server_::step() {
    // the records are read by poll() and the queue is fed by submit(): hold
    // the lock for the pass (the device calls below only enqueue work)
    std::lock_guard<std::mutex> lk(mu);
    bool progress = false;
    std::vector<Job *> finished;
    // 1. device work that completed
    for (Job *j : running) {
        if (!j->busy) continue;
        const hipError_t q = hipEventQuery(j->done);
        if (q == hipErrorNotReady) continue;
        progress = true;
        j->busy = false;
        if (q != hipSuccess) {
            fail(j, SS_E_DEVICE);
            finished.push_back(j);
            continue;
        }
        if (j->phase == kSweep) {
            j->cur ^= 1;
            j->info.steps_done += j->advance;
        } else if (j->phase == kCopyOut) {
            finished.push_back(j);
        }
    }
    // 2. jobs whose sweeps are done (or failed) copy their result out
    for (Job *j : running) {
        if (j->busy || j->phase == kCopyOut) continue;
        if (j->info.status != SS_OK) {
            if (std::find(finished.begin(), finished.end(), j) == finished.end()) finished.push_back(j);
            continue;
        }
        if (j->info.steps_done < j->info.steps_total) continue;
        hipStream_t st = stream_of(j->plan);
        if (hipMemcpyAsync(j->out, j->buf[j->cur], j->grid_bytes, hipMemcpyDefault, st) != hipSuccess ||
            hipEventRecord(j->done, st) != hipSuccess) {
            fail(j, SS_E_DEVICE);
            finished.push_back(j);
            continue;
        }
        j->phase = kCopyOut;
        j->busy = true;
        progress = true;
    }
    // 3. retire: free arena space and publish the record
    if (!finished.empty()) {
        const double t = now();
        for (Job *j : finished) {
            j->info.state = j->info.status == SS_OK ? 2 : 3;
            j->info.t_done = t;
            arena.release(j->arena_off);
            event_pool.push_back(j->done);
            j->done = nullptr;
            running.erase(std::find(running.begin(), running.end(), j));
            --live;
        }
        cv.notify_all();
    }
    // 4. admission, FIFO while the arena has room for both buffers
    {
        while (!queue.empty()) {
            Job *j = queue.front();
            size_t off;
            if (!arena.alloc(2 * round_up(j->grid_bytes), &off)) break;
            hipEvent_t e = take_event();
            if (!e) {
                arena.release(off);
                break;
            }
            queue.pop_front();
            j->arena_off = off;
            j->buf[0] = arena_base + off;
            j->buf[1] = arena_base + off + round_up(j->grid_bytes);
            j->cur = 0;
            j->done = e;
            j->info.state = 1;
            j->info.t_admit = now();
            running.push_back(j);
            hipStream_t st = stream_of(j->plan);
            if (hipMemcpyAsync(j->buf[0], j->in, j->grid_bytes, hipMemcpyDefault, st) != hipSuccess ||
                hipEventRecord(j->done, st) != hipSuccess) {
                j->info.status = SS_E_DEVICE;
            } else {
                j->phase = kCopyIn;
                j->busy = true;
            }
            progress = true;
        }
    }
    // 5. next sweep of every idle job, grouped by plan class (fused sweeps
    // and leftover single sweeps are different classes)
    std::vector<std::pair<const ss_plan_ *, std::vector<Job *>>> groups;
    for (Job *j : running) {
        if (j->busy || j->info.status != SS_OK || j->info.steps_done >= j->info.steps_total) continue;
        const int64_t left = j->info.steps_total - j->info.steps_done;
        const ss_plan_ *sub = (j->plan->fuse > 1 && left < j->plan->fuse) ? j->plan->rem : j->plan;
        auto g = std::find_if(groups.begin(), groups.end(), [&](const auto &e) {
            return e.second.size() < (size_t)ss::kMaxJobs && ss::same_class(e.first, sub);
        });
        if (g == groups.end()) groups.push_back({sub, {j}});
        else g->second.push_back(j);
    }
    for (auto &grp : groups) {
        const void *in[ss::kMaxJobs];
        void *out[ss::kMaxJobs];
        int64_t dims[ss::kMaxJobs][3];
        for (size_t t = 0; t < grp.second.size(); ++t) {
            Job *j = grp.second[t];
            in[t] = j->buf[j->cur];
            out[t] = j->buf[j->cur ^ 1];
            std::memcpy(dims[t], j->plan->dims, sizeof dims[t]);
        }
        hipStream_t st = stream_of(grp.first);
        bool ok = ss::sweep_grids(grp.first, (int)grp.second.size(), in, out, dims, st) == hipSuccess;
        // every job of the launch records its own event after it
        for (Job *j : grp.second) ok = ok && hipEventRecord(j->done, st) == hipSuccess;
        for (Job *j : grp.second) {
            if (!ok) {
                fail(j, SS_E_DEVICE);
                continue;
            }
            j->phase = kSweep;
            // the launched plan sets the sweeps (a job's own fused plan, or
            // an equal-class plan of another job, or a leftover single sweep)
            j->advance = grp.first->fuse;
            j->busy = true;
        }
        progress = true;
    }
    return progress;
}

void ss_server_::run() {
    (void)hipSetDevice(device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || !queue.empty() || !running.empty(); });
            if (stop && queue.empty() && running.empty()) break;
        }
        if (!step()) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    event_pool.clear();
}

extern "C" {

ss_status sparstencil_server_create(ss_server_t *out, void *arena, size_t arena_bytes, int32_t max_jobs,
                                    int32_t num_streams) {
    if (!out || !arena || arena_bytes == 0 || max_jobs < 1 || num_streams < 1 || num_streams > 16)
        return SS_E_INVALID;
    *out = nullptr;
    ss_server_ *s = new (std::nothrow) ss_server_(arena_bytes);
    if (!s) return SS_E_NOMEM;
    s->arena_base = static_cast<char *>(arena);
    s->max_jobs = max_jobs;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return SS_E_DEVICE;
    }
    for (int i = 0; i < num_streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return SS_E_DEVICE;
        }
        s->streams.push_back(st);
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return SS_OK;
}

ss_status sparstencil_submit(ss_server_t s, ss_plan_t plan, const void *in, void *out, int64_t steps,
                             uint64_t *job_id) {
    if (!s || !plan || !in || !out || steps < 1 || !job_id || plan->host_only) return SS_E_INVALID;
    const size_t bytes = sparstencil_grid_bytes(plan);
    // a job whose two buffers exceed the whole arena could never be admitted
    if (2 * round_up(bytes) > s->arena_bytes) return SS_E_NOMEM;
    Job *j = new (std::nothrow) Job();
    if (!j) return SS_E_NOMEM;
    j->plan = plan;
    j->in = in;
    j->out = out;
    j->grid_bytes = bytes;
    j->info.steps_total = steps;
    j->info.status = SS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop || s->live >= s->max_jobs) {
            delete j;
            return s->stop ? SS_E_INVALID : SS_E_BUSY;
        }
        j->info.id = s->next_id++;
        j->info.t_submit = s->now();
        s->jobs[j->info.id] = j;
        s->queue.push_back(j);
        ++s->live;
        *job_id = j->info.id;
    }
    s->cv.notify_all();
    return SS_OK;
}

ss_status sparstencil_poll(ss_server_t s, uint64_t job_id, ss_job_info *info) {
    if (!s) return SS_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return SS_E_NOT_FOUND;
    if (info) *info = it->second->info;
    const int st = it->second->info.state;
    if (st == 3) return (ss_status)it->second->info.status;
    return st == 2 ? SS_OK : SS_PENDING;
}

ss_status sparstencil_job_release(ss_server_t s, uint64_t job_id) {
    if (!s) return SS_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return SS_E_NOT_FOUND;
    if (it->second->info.state < 2) return SS_E_BUSY;
    delete it->second;
    s->jobs.erase(it);
    return SS_OK;
}

ss_status sparstencil_server_drain(ss_server_t s) {
    if (!s) return SS_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->live == 0; });
    return SS_OK;
}

double sparstencil_server_clock(ss_server_t s) { return s ? s->now() : 0.0; }

ss_status sparstencil_server_destroy(ss_server_t s) {
    if (!s) return SS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    for (auto &e : s->jobs) delete e.second;
    delete s;
    return SS_OK;
}

}  // extern "C"
