// Serving loop: continuous batching of reconstruction jobs on one device.
//
// A background thread keeps up to `max_slots` launches in flight, each on its
// own stream.  A job is cut into pieces of at most kPiece patches, so that
// the copies in and out of one piece overlap the kernels of the others and a
// large job spreads over several slots.  Pieces wait in arrival order; when a
// slot is free and the head piece's device buffers fit in the HBM budget, the
// head piece and the pieces queued right behind it that share its plan and
// its kind (zero-tree or full OMP, same coarse sparsities) are packed into
// one launch, up to kPiece patches.  Each launch copies its pieces' host
// inputs into fresh device buffers, runs cspd_omp_cross_scale /
// cspd_omp_full over the packed batch, copies every piece's rows back to its
// job's host buffers and records an event; the thread retires launches whose
// events have completed and returns their memory to the budget.  A job is
// finished when its last piece is.  A patch's result does not depend on the
// other patches of a launch, so a job gives the same result alone, in a mix
// and cut into pieces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cspd_internal.h"

using namespace cspd;

namespace {

constexpr int64_t kPiece = 1 << 16;   // patches per piece and per launch

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Job {
    cspd_job d{};
    uint64_t id = 0;
    cspd_job_stats st{};
    int pieces_left = 0;
    bool admitted = false;
    bool started = false;
    bool done = false;
};

// Rows [row, row + b) of one job.
struct Piece {
    Job *job = nullptr;
    int64_t row = 0;
    int64_t b = 0;
    int64_t bytes = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<Piece> pieces;
    int64_t bytes = 0;
    int status = CSPD_OK;
    int32_t *kbuf = nullptr;   // pinned: per-patch K of the packed batch (kept until retired)
    char *dev = nullptr;       // device buffers of a launch, kept and grown (never shrunk)
    size_t dev_bytes = 0;
};

size_t esize(const cspd_plan_s *p) { return p->dtype == CSPD_F64 ? sizeof(double) : sizeof(float); }

// Device bytes one job's patches occupy in a launch (inputs + outputs).
int64_t job_bytes(const cspd_plan_s *p, int64_t B)
{
    const int64_t e = (int64_t)esize(p);
    int64_t per = e * p->m + sizeof(int32_t)                      // y, k
                  + (int64_t)p->k_max * (sizeof(int32_t) + e)       // support, coef
                  + sizeof(int32_t) + e * p->n;                     // k_used, xhat
    if (p->phi_kind == CSPD_PHI_MASK) per += p->n;
    int64_t coarse = 0;
    for (int s = 0; s + 1 < p->s; ++s) coarse += p->k_max;
    per += coarse * (int64_t)sizeof(int32_t);
    per += cross_workspace_per_patch(p);   // the call's own workspace
    return per * B + 4096;
}

bool same_batch(const Job *a, const Job *b)
{
    if (a == b) return true;
    if (a->d.plan != b->d.plan || a->d.full != b->d.full) return false;
    if (a->d.full) return true;
    for (int s = 0; s + 1 < a->d.plan->s; ++s)
        if (a->d.k_scale[s] != b->d.k_scale[s]) return false;
    return true;
}

}  // namespace

struct cspd_server_s {
    int device = 0;
    int64_t budget = 0;
    int64_t used = 0;
    int max_slots = 1;
    uint64_t next_id = 1;
    std::mutex mu;
    std::condition_variable wake;   // scheduler
    std::condition_variable fin;    // pollers
    std::deque<Piece> queue;
    std::unordered_map<uint64_t, Job *> jobs;
    std::vector<Slot> slots;
    std::thread worker;
    bool stop = false;

    void run();
    bool retire_locked();
    bool take_locked(Slot &sl);
    void enqueue(Slot &sl);
};

// Pop the head piece and the compatible pieces queued behind it into a free
// slot (lock held).  Returns false when nothing can be admitted now.
bool cspd_server_s::take_locked(Slot &sl)
{
    if (queue.empty()) return false;
    const Piece &head = queue.front();
    if (used + head.bytes > budget) return false;   // wait for memory (arrival order is kept)
    size_t n = 1;
    int64_t bytes = head.bytes, patches = head.b;
    for (; n < queue.size(); ++n) {
        const Piece &q = queue[n];
        if (!same_batch(head.job, q.job)) break;
        if (patches + q.b > kPiece || used + bytes + q.bytes > budget) break;
        bytes += q.bytes;
        patches += q.b;
    }
    sl.pieces.assign(queue.begin(), queue.begin() + (long)n);
    queue.erase(queue.begin(), queue.begin() + (long)n);
    used += bytes;
    const int64_t t_admit = now_ns();
    int jobs_here = 0;
    for (size_t i = 0; i < n; ++i)
        if (i == 0 || sl.pieces[i].job != sl.pieces[i - 1].job) ++jobs_here;
    for (Piece &q : sl.pieces) {
        Job *jb = q.job;
        if (!jb->admitted) {
            jb->admitted = true;
            jb->st.admit_ns = t_admit;
        }
        if (jobs_here - 1 > jb->st.batched_with) jb->st.batched_with = jobs_here - 1;
    }
    sl.bytes = bytes;
    sl.busy = true;
    sl.status = CSPD_OK;
    return true;
}

// Copy in, launch and copy out one packed batch (lock not held; only the
// scheduler thread touches slots and the started flags).
void cspd_server_s::enqueue(Slot &sl)
{
    const std::vector<Piece> &take = sl.pieces;
    const Job *head = take.front().job;
    int64_t patches = 0;
    for (const Piece &q : take) patches += q.b;
    cspd_plan_s *p = head->d.plan;
    const int64_t B = patches;
    const size_t e = esize(p);
    int ks = 0;
    for (int s = 0; s + 1 < p->s; ++s) ks += head->d.k_scale[s];
    // carve the launch's buffers out of one stream-ordered allocation
    size_t off = 0;
    auto carve = [&](size_t n) { size_t o = off; off += (n + 255) / 256 * 256; return o; };
    const size_t o_y = carve(e * (size_t)B * p->m);
    const size_t o_m = carve(p->phi_kind == CSPD_PHI_MASK ? (size_t)B * p->n : 0);
    const size_t o_k = carve(sizeof(int32_t) * (size_t)B);
    const size_t o_sup = carve(sizeof(int32_t) * (size_t)B * p->k_max);
    const size_t o_cf = carve(e * (size_t)B * p->k_max);
    const size_t o_ku = carve(sizeof(int32_t) * (size_t)B);
    const size_t o_x = carve(e * (size_t)B * p->n);
    const size_t o_sc = carve(sizeof(int32_t) * (size_t)B * (ks > 0 ? ks : 1));
    const size_t wbytes = head->d.full ? 0 : cross_call_workspace(p, B, head->d.k_scale, true);
    const size_t o_ws = carve(wbytes);
    int rc = CSPD_OK;
    // the slot's buffers are reused launch after launch (this slot's previous
    // launch has retired, so its stream is idle); they grow when a launch
    // needs more, with a synchronous allocation that only the first launches
    // of each size pay
    if (sl.dev_bytes < off) {
        if (sl.dev) (void)hipFree(sl.dev);
        sl.dev = nullptr;
        sl.dev_bytes = 0;
        if (hipMalloc((void **)&sl.dev, off) == hipSuccess) sl.dev_bytes = off;
        else rc = CSPD_E_NOMEM;
    }
    char *dev = sl.dev;
    const int64_t t_start = now_ns();
    int32_t *kbuf = sl.kbuf;
    if (rc == CSPD_OK) {
        int64_t row = 0;
        for (const Piece &q : take) {
            Job *j = q.job;
            if (!j->started) {
                j->started = true;
                j->st.start_ns = t_start;
            }
            const int64_t b = q.b;
            hipMemcpyAsync(dev + o_y + e * (size_t)row * p->m, (const char *)j->d.y + e * (size_t)q.row * p->m,
                           e * (size_t)b * p->m, hipMemcpyHostToDevice, sl.stream);
            if (p->phi_kind == CSPD_PHI_MASK)
                hipMemcpyAsync(dev + o_m + (size_t)row * p->n, j->d.mask + (size_t)q.row * p->n, (size_t)b * p->n,
                               hipMemcpyHostToDevice, sl.stream);
            for (int64_t i = 0; i < b; ++i)
                kbuf[row + i] = j->d.k_fine ? j->d.k_fine[q.row + i] : j->d.k_fine_uniform;
            row += b;
        }
        hipMemcpyAsync(dev + o_k, kbuf, sizeof(int32_t) * (size_t)B, hipMemcpyHostToDevice, sl.stream);
        if (head->d.full)
            rc = cspd_omp_full(p, B, dev + o_y, (const uint8_t *)(dev + o_m), (const int32_t *)(dev + o_k), 0,
                               (int32_t *)(dev + o_sup), dev + o_cf, (int32_t *)(dev + o_ku), dev + o_x,
                               sl.stream);
        else
            rc = cross_scale_on(p, B, dev + o_y, (const uint8_t *)(dev + o_m), head->d.k_scale,
                                (const int32_t *)(dev + o_k), 0, (int32_t *)(dev + o_sup), dev + o_cf,
                                (int32_t *)(dev + o_ku), dev + o_x, (int32_t *)(dev + o_sc), dev + o_ws, wbytes,
                                sl.stream);
        row = 0;
        for (const Piece &q : take) {
            const Job *j = q.job;
            const int64_t b = q.b;
            const size_t r = (size_t)q.row;
            if (rc == CSPD_OK) {
                hipMemcpyAsync(j->d.support + r * p->k_max, dev + o_sup + sizeof(int32_t) * (size_t)row * p->k_max,
                               sizeof(int32_t) * (size_t)b * p->k_max, hipMemcpyDeviceToHost, sl.stream);
                hipMemcpyAsync(j->d.k_used + r, dev + o_ku + sizeof(int32_t) * (size_t)row,
                               sizeof(int32_t) * (size_t)b, hipMemcpyDeviceToHost, sl.stream);
                if (j->d.coef)
                    hipMemcpyAsync((char *)j->d.coef + e * r * p->k_max, dev + o_cf + e * (size_t)row * p->k_max,
                                   e * (size_t)b * p->k_max, hipMemcpyDeviceToHost, sl.stream);
                if (j->d.xhat)
                    hipMemcpyAsync((char *)j->d.xhat + e * r * p->n, dev + o_x + e * (size_t)row * p->n,
                                   e * (size_t)b * p->n, hipMemcpyDeviceToHost, sl.stream);
            }
            row += b;
        }
    }
    sl.status = rc;
    hipEventRecord(sl.ev, sl.stream);
}

// Retire finished launches (lock held).  Returns true if any finished.
bool cspd_server_s::retire_locked()
{
    bool any = false;
    for (Slot &sl : slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.ev);
        if (q == hipErrorNotReady) continue;
        const int status = q == hipSuccess ? sl.status : CSPD_E_DEVICE;
        const int64_t t = now_ns();
        for (Piece &pc : sl.pieces) {
            Job *j = pc.job;
            if (status != CSPD_OK && j->st.status == CSPD_OK) j->st.status = status;
            if (--j->pieces_left == 0) {
                j->st.finish_ns = t;
                j->done = true;
            }
        }
        used -= sl.bytes;
        sl.pieces.clear();
        sl.bytes = 0;
        sl.busy = false;
        any = true;
    }
    return any;
}

void cspd_server_s::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        const bool retired = retire_locked();
        if (retired) fin.notify_all();
        bool launched = false;
        for (Slot &sl : slots) {
            if (sl.busy || !take_locked(sl)) continue;
            lk.unlock();
            enqueue(sl);
            lk.lock();
            launched = true;
        }
        bool in_flight = false;
        for (Slot &sl : slots) in_flight |= sl.busy;
        if (stop && queue.empty() && !in_flight) break;
        if (launched || retired) continue;
        // sleep until a submission arrives or, with launches in flight, briefly
        if (in_flight) wake.wait_for(lk, std::chrono::microseconds(50));
        else wake.wait_for(lk, std::chrono::milliseconds(20));
    }
    fin.notify_all();
}

extern "C" {

cspd_status cspd_serve_create(int32_t device, int64_t hbm_budget_bytes, int32_t max_slots, cspd_server_t *out)
{
    clear_error();
    if (!out) return set_error(CSPD_E_INVALID, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes <= 0) return set_error(CSPD_E_INVALID, "hbm budget %lld", (long long)hbm_budget_bytes);
    if (max_slots < 1 || max_slots > 64) return set_error(CSPD_E_INVALID, "max_slots %d outside 1..64", max_slots);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return set_error(CSPD_E_DEVICE, "device %d not available", device);
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return set_error(CSPD_E_DEVICE, "hipSetDevice(%d)", device);
    cspd_server_s *s = new (std::nothrow) cspd_server_s();
    if (!s) return set_error(CSPD_E_NOMEM, "host allocation failed");
    s->device = device;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->slots.resize((size_t)max_slots);
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&sl.kbuf, sizeof(int32_t) * kPiece, hipHostMallocDefault) != hipSuccess) {
            for (Slot &x : s->slots) {
                if (x.stream) (void)hipStreamDestroy(x.stream);
                if (x.ev) (void)hipEventDestroy(x.ev);
                if (x.kbuf) (void)hipHostFree(x.kbuf);
            }
            delete s;
            (void)hipSetDevice(prev);
            return set_error(CSPD_E_DEVICE, "stream or event creation failed");
        }
    }
    (void)hipSetDevice(prev);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return CSPD_OK;
}

cspd_status cspd_serve_submit(cspd_server_t s, const cspd_job *job, uint64_t *job_id)
{
    clear_error();
    if (!s || !job || !job_id) return set_error(CSPD_E_INVALID, "NULL argument");
    const cspd_plan_s *p = job->plan;
    if (!p) return set_error(CSPD_E_INVALID, "job without plan");
    if (p->device != s->device) return set_error(CSPD_E_INVALID, "plan lives on device %d, server on %d", p->device, s->device);
    if (job->B < 0) return set_error(CSPD_E_INVALID, "B = %lld", (long long)job->B);
    if (job->B > 0 && (!job->y || !job->support || !job->k_used))
        return set_error(CSPD_E_INVALID, "y / support / k_used is NULL");
    if (job->B > 0 && p->phi_kind == CSPD_PHI_MASK && !job->mask) return set_error(CSPD_E_INVALID, "mask plan needs a mask");
    if (p->n_phases > 1) return set_error(CSPD_E_INVALID, "plan has %d operators: not served", p->n_phases);
    if (!job->k_fine && (job->k_fine_uniform < 0 || job->k_fine_uniform > p->k_max))
        return set_error(CSPD_E_SHAPE, "k_fine_uniform %d outside [0, %d]", job->k_fine_uniform, p->k_max);
    if (!job->full)
        for (int i = 0; i + 1 < p->s; ++i)
            if (job->k_scale[i] < 0 || job->k_scale[i] > p->k_max)
                return set_error(CSPD_E_SHAPE, "k_scale[%d] = %d outside [0, %d]", i, job->k_scale[i], p->k_max);
    if (job->k_fine)
        for (int64_t i = 0; i < job->B; ++i)
            if (job->k_fine[i] < 0 || job->k_fine[i] > p->k_max)
                return set_error(CSPD_E_SHAPE, "k_fine[%lld] = %d outside [0, %d]", (long long)i, job->k_fine[i], p->k_max);
    const int64_t bytes = job_bytes(p, job->B < kPiece ? job->B : kPiece);
    if (bytes > s->budget)
        return set_error(CSPD_E_CAPACITY, "a piece of the job needs %lld bytes, budget is %lld", (long long)bytes,
                         (long long)s->budget);
    Job *j = new (std::nothrow) Job();
    if (!j) return set_error(CSPD_E_NOMEM, "host allocation failed");
    j->d = *job;
    j->st.patches = job->B;
    j->st.submit_ns = now_ns();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) { delete j; return set_error(CSPD_E_INVALID, "server is shutting down"); }
        j->id = s->next_id++;
        s->jobs[j->id] = j;
        if (job->B == 0) {
            j->st.admit_ns = j->st.start_ns = j->st.finish_ns = j->st.submit_ns;
            j->done = true;
        } else {
            for (int64_t r = 0; r < job->B; r += kPiece) {
                Piece q;
                q.job = j;
                q.row = r;
                q.b = job->B - r < kPiece ? job->B - r : kPiece;
                q.bytes = job_bytes(p, q.b);
                s->queue.push_back(q);
                ++j->pieces_left;
            }
        }
        *job_id = j->id;
    }
    s->wake.notify_one();
    return CSPD_OK;
}

cspd_status cspd_serve_poll(cspd_server_t s, uint64_t job_id, int64_t timeout_us, cspd_job_stats *stats)
{
    clear_error();
    if (!s) return set_error(CSPD_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return set_error(CSPD_E_NOTFOUND, "job %llu unknown", (unsigned long long)job_id);
    Job *j = it->second;
    if (!j->done && timeout_us != 0) {
        auto pred = [j] { return j->done; };
        if (timeout_us < 0) s->fin.wait(lk, pred);
        else s->fin.wait_for(lk, std::chrono::microseconds(timeout_us), pred);
    }
    if (!j->done) return CSPD_E_BUSY;
    if (stats) *stats = j->st;
    const int status = j->st.status;
    s->jobs.erase(it);
    delete j;
    if (status != CSPD_OK) return set_error(status, "job %llu failed", (unsigned long long)job_id);
    return CSPD_OK;
}

void cspd_serve_destroy(cspd_server_t s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->wake.notify_all();
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.kbuf) (void)hipHostFree(sl.kbuf);
        if (sl.dev) (void)hipFree(sl.dev);
    }
    (void)hipSetDevice(prev);
    for (auto &kv : s->jobs) delete kv.second;
    delete s;
}

}  // extern "C"
