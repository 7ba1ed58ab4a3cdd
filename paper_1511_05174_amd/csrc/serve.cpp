// Serving loop: continuous batching of reconstruction jobs on one device.
//
// A background thread keeps up to `max_slots` launches in flight, each on its
// own stream.  A job is cut into pieces of at most kPiece patches, so that
// the copies in and out of one piece overlap the kernels of the others and a
// large job spreads over several slots.  When a slot is free, the scheduler
// picks a piece -- the oldest piece of a small job (at most kSmall patches)
// while the oldest waiting piece has waited less than kMaxWaitNs, else the
// oldest piece -- and packs the waiting pieces that share its plan and its
// kind (zero-tree or full OMP, same coarse sparsities) into one launch, up to
// kPiece patches.  With two or more slots, large pieces never take the last
// free slot, so a small job does not wait behind large jobs' copies.  A launch
// of host-buffer jobs copies its pieces' inputs into the slot's device
// buffers, runs cspd_omp_cross_scale / cspd_omp_full over the packed batch,
// copies every piece's rows back to its job's host buffers and records an
// event; a piece of a device-buffer job runs in place on the job's own
// buffers (nothing to copy, not packed).  The thread retires launches whose
// events have completed.  A job is finished when its last piece is.  A
// patch's result does not depend on the other patches of a launch, so a job
// gives the same result alone, in a mix and cut into pieces.
//
// HBM budget: every byte the server holds on the device counts -- each slot
// keeps its buffers from launch to launch (grown to its largest launch), in
// flight or idle.  A launch that would take the total past the budget first
// releases idle slots' buffers, else waits for memory.  No C++ exception
// leaves the library: the entry points and the scheduler thread catch them
// and turn them into statuses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <mutex>
#include <new>
#include <system_error>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cspd_internal.h"

using namespace cspd;

namespace {

constexpr int64_t kPiece = 1 << 16;         // patches per piece and per launch
constexpr int64_t kSmall = 8192;            // jobs of at most this many patches go first ...
constexpr int64_t kMaxWaitNs = 5000000;     // ... while the oldest piece has waited less than this

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
    bool small = false;
    bool admitted = false;
    bool started = false;
    bool done = false;
};

// Rows [row, row + b) of one job.
struct Piece {
    Job *job = nullptr;
    int64_t row = 0;
    int64_t b = 0;
    int64_t enq_ns = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<Piece> pieces;
    int status = CSPD_OK;
    int32_t *kbuf = nullptr;   // pinned: per-patch K of the packed batch (kept until retired)
    char *dev = nullptr;       // the slot's device buffers, reused launch after launch
    size_t dev_bytes = 0;      // allocated
    size_t cap = 0;            // reserved against the budget (>= dev_bytes; > while a growth is pending)
};

size_t esize(const cspd_plan_s *p) { return p->dtype == CSPD_F64 ? sizeof(double) : sizeof(float); }

// Device buffers of one launch of B patches: host-buffer jobs need inputs,
// outputs, coarse supports and the call's workspace; device-buffer jobs only
// the workspace (which then also holds the coarse supports).
struct Layout {
    size_t y = 0, m = 0, k = 0, sup = 0, cf = 0, ku = 0, x = 0, sc = 0, ws = 0;
    size_t wbytes = 0, total = 0;
};

Layout layout(const cspd_plan_s *p, int64_t B, const cspd_job &d)
{
    Layout L;
    size_t off = 0;
    auto carve = [&](size_t n) { size_t o = off; off += (n + 255) / 256 * 256; return o; };
    const size_t e = esize(p), b = (size_t)B;
    if (!d.on_device) {
        int ks = 0;
        for (int s = 0; s + 1 < p->s; ++s) ks += d.k_scale[s];
        L.y = carve(e * b * p->m);
        L.m = carve(p->phi_kind == CSPD_PHI_MASK ? b * p->n : 0);
        L.k = carve(sizeof(int32_t) * b);
        L.sup = carve(sizeof(int32_t) * b * p->k_max);
        L.cf = carve(e * b * p->k_max);
        L.ku = carve(sizeof(int32_t) * b);
        L.x = carve(e * b * p->n);
        L.sc = carve(sizeof(int32_t) * b * (ks > 0 ? ks : 1));
    }
    L.wbytes = d.full ? 0 : cross_call_workspace(p, B, d.k_scale, !d.on_device);
    L.ws = carve(L.wbytes);
    L.total = off;
    return L;
}

bool same_batch(const Job *a, const Job *b)
{
    if (a->d.on_device || b->d.on_device) return false;   // run in place, one piece per launch
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
    int64_t resident = 0;      // sum of the slots' reserved bytes
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
    int fatal = CSPD_OK;            // set if the scheduler thread failed

    void run();
    void run_loop();
    bool retire_locked();
    bool take_locked(Slot &sl);
    bool fits_locked(Slot &sl, size_t need);
    void enqueue(Slot &sl);
    void fail_all_locked(int status);
};

// Whether slot sl can hold `need` bytes within the budget, releasing idle
// slots' buffers if that makes it fit (lock held; only the scheduler thread
// touches slots, and an idle slot's stream has nothing pending).
bool cspd_server_s::fits_locked(Slot &sl, size_t need)
{
    auto total = [&] { return resident - (int64_t)sl.cap + (int64_t)std::max(sl.cap, need); };
    if (total() <= budget) return true;
    for (Slot &x : slots) {
        if (&x == &sl || x.busy || x.cap == 0) continue;
        if (x.dev) (void)hipFree(x.dev);
        resident -= (int64_t)x.cap;
        x.dev = nullptr;
        x.dev_bytes = 0;
        x.cap = 0;
        if (total() <= budget) return true;
    }
    return total() <= budget;
}

// Pick a piece, pack the compatible waiting pieces with it into a free slot
// and reserve its memory (lock held).  Returns false when nothing can be
// admitted now.
bool cspd_server_s::take_locked(Slot &sl)
{
    if (queue.empty()) return false;
    const int64_t t_now = now_ns();
    constexpr size_t kNone = ~(size_t)0;
    // with three or more slots, large pieces leave the last free slot to small jobs
    int free_slots = 0;
    for (const Slot &x : slots) free_slots += !x.busy;
    const bool large_ok = max_slots < 3 || free_slots >= 2;
    size_t first_small = kNone;
    for (size_t i = 0; i < queue.size(); ++i)
        if (queue[i].job->small) { first_small = i; break; }
    const bool aged = t_now - queue.front().enq_ns >= kMaxWaitNs;
    size_t h = aged ? (large_ok ? 0 : first_small) : (first_small != kNone ? first_small : (large_ok ? 0 : kNone));
    if (h == kNone) return false;
    const Piece &head = queue[h];
    const cspd_plan_s *p = head.job->d.plan;
    std::vector<size_t> pick{h};
    int64_t patches = head.b;
    size_t need = layout(p, patches, head.job->d).total;
    if (!fits_locked(sl, need)) return false;   // wait for memory
    // pack the compatible waiting pieces in queue order; a job whose piece is
    // passed over keeps its later pieces waiting too (pieces keep their order)
    std::vector<const Job *> passed;
    constexpr size_t kScan = 1024;   // queue entries looked at per launch
    for (size_t i = 0; i < queue.size() && i < kScan && patches < kPiece; ++i) {
        if (i == h) continue;
        const Piece &q = queue[i];
        const bool blocked = std::find(passed.begin(), passed.end(), q.job) != passed.end();
        bool ok = !blocked && same_batch(head.job, q.job) && patches + q.b <= kPiece;
        size_t n2 = 0;
        if (ok) {
            n2 = layout(p, patches + q.b, head.job->d).total;
            ok = fits_locked(sl, n2);
        }
        if (!ok) {
            if (!blocked) passed.push_back(q.job);
            continue;
        }
        pick.push_back(i);
        patches += q.b;
        need = n2;
    }
    std::sort(pick.begin(), pick.end());
    sl.pieces.clear();
    for (size_t i : pick) sl.pieces.push_back(queue[i]);
    for (size_t k = pick.size(); k-- > 0;) queue.erase(queue.begin() + (long)pick[k]);
    if (need > sl.cap) {
        resident += (int64_t)(need - sl.cap);
        sl.cap = need;
    }
    int jobs_here = 0;
    for (size_t i = 0; i < sl.pieces.size(); ++i)
        if (i == 0 || sl.pieces[i].job != sl.pieces[i - 1].job) ++jobs_here;
    for (Piece &q : sl.pieces) {
        Job *jb = q.job;
        if (!jb->admitted) {
            jb->admitted = true;
            jb->st.admit_ns = t_now;
        }
        if (jobs_here - 1 > jb->st.batched_with) jb->st.batched_with = jobs_here - 1;
    }
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
    const Layout L = layout(p, B, head->d);
    int rc = CSPD_OK;
    auto chk = [&](hipError_t r) { if (r != hipSuccess && rc == CSPD_OK) rc = CSPD_E_DEVICE; };
    // the slot's buffers are reused launch after launch (this slot's previous
    // launch has retired, so its stream is idle); they grow to the reserved
    // size when a launch needs more, with a synchronous allocation that only
    // the first launches of each size pay
    if (sl.dev_bytes < L.total) {
        if (sl.dev) (void)hipFree(sl.dev);
        sl.dev = nullptr;
        sl.dev_bytes = 0;
        if (hipMalloc((void **)&sl.dev, sl.cap) == hipSuccess) sl.dev_bytes = sl.cap;
        else rc = CSPD_E_NOMEM;
    }
    char *dev = sl.dev;
    const int64_t t_start = now_ns();
    for (const Piece &q : take) {
        Job *j = q.job;
        if (!j->started) {
            j->started = true;
            j->st.start_ns = t_start;
        }
    }
    if (rc == CSPD_OK && head->d.on_device) {
        // one piece of a device-buffer job, in place
        const Piece &q = take.front();
        const cspd_job &d = q.job->d;
        const size_t r = (size_t)q.row;
        const void *y = (const char *)d.y + e * r * p->m;
        const uint8_t *mask = d.mask ? d.mask + r * p->n : nullptr;
        const int32_t *kf = d.k_fine ? d.k_fine + r : nullptr;
        int32_t *sup = d.support + r * p->k_max;
        void *cf = d.coef ? (char *)d.coef + e * r * p->k_max : nullptr;
        int32_t *ku = d.k_used + r;
        void *xh = d.xhat ? (char *)d.xhat + e * r * p->n : nullptr;
        if (d.full)
            rc = cspd_omp_full(p, q.b, y, mask, kf, d.k_fine_uniform, sup, cf, ku, xh, sl.stream);
        else
            rc = cross_scale_on(p, q.b, y, mask, d.k_scale, kf, d.k_fine_uniform, sup, cf, ku, xh, nullptr,
                                dev + L.ws, L.wbytes, sl.stream);
    } else if (rc == CSPD_OK) {
        int32_t *kbuf = sl.kbuf;
        int64_t row = 0;
        for (const Piece &q : take) {
            const Job *j = q.job;
            const int64_t b = q.b;
            chk(hipMemcpyAsync(dev + L.y + e * (size_t)row * p->m, (const char *)j->d.y + e * (size_t)q.row * p->m,
                               e * (size_t)b * p->m, hipMemcpyHostToDevice, sl.stream));
            if (p->phi_kind == CSPD_PHI_MASK)
                chk(hipMemcpyAsync(dev + L.m + (size_t)row * p->n, j->d.mask + (size_t)q.row * p->n,
                                   (size_t)b * p->n, hipMemcpyHostToDevice, sl.stream));
            for (int64_t i = 0; i < b; ++i)
                kbuf[row + i] = j->d.k_fine ? j->d.k_fine[q.row + i] : j->d.k_fine_uniform;
            row += b;
        }
        chk(hipMemcpyAsync(dev + L.k, kbuf, sizeof(int32_t) * (size_t)B, hipMemcpyHostToDevice, sl.stream));
        if (rc == CSPD_OK) {
            if (head->d.full)
                rc = cspd_omp_full(p, B, dev + L.y, (const uint8_t *)(dev + L.m), (const int32_t *)(dev + L.k), 0,
                                   (int32_t *)(dev + L.sup), dev + L.cf, (int32_t *)(dev + L.ku), dev + L.x,
                                   sl.stream);
            else
                rc = cross_scale_on(p, B, dev + L.y, (const uint8_t *)(dev + L.m), head->d.k_scale,
                                    (const int32_t *)(dev + L.k), 0, (int32_t *)(dev + L.sup), dev + L.cf,
                                    (int32_t *)(dev + L.ku), dev + L.x, (int32_t *)(dev + L.sc), dev + L.ws,
                                    L.wbytes, sl.stream);
        }
        row = 0;
        for (const Piece &q : take) {
            const Job *j = q.job;
            const int64_t b = q.b;
            const size_t r = (size_t)q.row;
            if (rc == CSPD_OK) {
                chk(hipMemcpyAsync(j->d.support + r * p->k_max, dev + L.sup + sizeof(int32_t) * (size_t)row * p->k_max,
                                   sizeof(int32_t) * (size_t)b * p->k_max, hipMemcpyDeviceToHost, sl.stream));
                chk(hipMemcpyAsync(j->d.k_used + r, dev + L.ku + sizeof(int32_t) * (size_t)row,
                                   sizeof(int32_t) * (size_t)b, hipMemcpyDeviceToHost, sl.stream));
                if (j->d.coef)
                    chk(hipMemcpyAsync((char *)j->d.coef + e * r * p->k_max, dev + L.cf + e * (size_t)row * p->k_max,
                                       e * (size_t)b * p->k_max, hipMemcpyDeviceToHost, sl.stream));
                if (j->d.xhat)
                    chk(hipMemcpyAsync((char *)j->d.xhat + e * r * p->n, dev + L.x + e * (size_t)row * p->n,
                                       e * (size_t)b * p->n, hipMemcpyDeviceToHost, sl.stream));
            }
            row += b;
        }
    }
    sl.status = rc;
    chk(hipEventRecord(sl.ev, sl.stream));
    if (rc != CSPD_OK) sl.status = rc;
}

// Retire finished launches (lock held).  Returns true if any finished.
bool cspd_server_s::retire_locked()
{
    bool any = false;
    for (Slot &sl : slots) {
        if (!sl.busy) continue;
        // a launch whose event was never recorded (status already failed) is
        // finished once its stream is idle
        hipError_t q = hipEventQuery(sl.ev);
        if (sl.status != CSPD_OK && q != hipSuccess) q = hipStreamQuery(sl.stream);
        if (q == hipErrorNotReady) continue;
        const int status = q == hipSuccess ? sl.status : CSPD_E_DEVICE;
        const int64_t t = now_ns();
        for (Piece &pc : sl.pieces) {
            Job *j = pc.job;
            if (status != CSPD_OK && j->st.status == CSPD_OK) j->st.status = status;
            if (--j->pieces_left == 0) {
                j->st.finish_ns = t;
                j->st.server_resident_bytes = resident;
                j->done = true;
            }
        }
        if (sl.dev_bytes < sl.cap) {   // the growth was not allocated: return the reservation
            resident -= (int64_t)(sl.cap - sl.dev_bytes);
            sl.cap = sl.dev_bytes;
        }
        sl.pieces.clear();
        sl.busy = false;
        any = true;
    }
    return any;
}

// The scheduler failed outside any launch: every waiting job fails with
// `status` (lock held).
void cspd_server_s::fail_all_locked(int status)
{
    fatal = status;
    for (Piece &q : queue) {
        Job *j = q.job;
        if (j->st.status == CSPD_OK) j->st.status = status;
        if (--j->pieces_left == 0) {
            j->st.finish_ns = now_ns();
            j->done = true;
        }
    }
    queue.clear();
}

void cspd_server_s::run_loop()
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
        else wake.wait_for(lk, std::chrono::milliseconds(queue.empty() ? 20 : 1));
    }
}

void cspd_server_s::run()
{
    try {
        run_loop();
    } catch (...) {
        // host memory ran out (or another C++ failure) in the scheduler:
        // launches in flight finish on their streams; queued jobs fail
        std::lock_guard<std::mutex> g(mu);
        for (Slot &sl : slots)
            if (sl.busy) (void)hipStreamSynchronize(sl.stream);
        for (Slot &sl : slots) {
            if (!sl.busy) continue;
            for (Piece &pc : sl.pieces) {
                Job *j = pc.job;
                if (--j->pieces_left == 0) {
                    j->st.finish_ns = now_ns();
                    j->done = true;
                }
            }
            sl.pieces.clear();
            sl.busy = false;
        }
        fail_all_locked(CSPD_E_NOMEM);
    }
    fin.notify_all();
}

extern "C" {

cspd_status cspd_serve_create(int32_t device, int64_t hbm_budget_bytes, int32_t max_slots, cspd_server_t *out)
{
    return guarded([&]() -> cspd_status {
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
    });
}

cspd_status cspd_serve_submit(cspd_server_t s, const cspd_job *job, uint64_t *job_id)
{
    return guarded([&]() -> cspd_status {
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
        if (job->k_fine && !job->on_device)   // device values are clamped by the kernels
            for (int64_t i = 0; i < job->B; ++i)
                if (job->k_fine[i] < 0 || job->k_fine[i] > p->k_max)
                    return set_error(CSPD_E_SHAPE, "k_fine[%lld] = %d outside [0, %d]", (long long)i, job->k_fine[i], p->k_max);
        const int64_t bytes = (int64_t)layout(p, job->B < kPiece ? job->B : kPiece, *job).total;
        if (bytes > s->budget)
            return set_error(CSPD_E_CAPACITY, "a piece of the job needs %lld bytes, budget is %lld", (long long)bytes,
                             (long long)s->budget);
        Job *j = new (std::nothrow) Job();
        if (!j) return set_error(CSPD_E_NOMEM, "host allocation failed");
        j->d = *job;
        j->small = job->B <= kSmall;
        j->st.patches = job->B;
        j->st.submit_ns = now_ns();
        {
            std::lock_guard<std::mutex> g(s->mu);
            if (s->stop) { delete j; return set_error(CSPD_E_INVALID, "server is shutting down"); }
            if (s->fatal != CSPD_OK) { delete j; return set_error(s->fatal, "the server's scheduler failed"); }
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
                    q.enq_ns = j->st.submit_ns;
                    s->queue.push_back(q);
                    ++j->pieces_left;
                }
            }
            *job_id = j->id;
        }
        s->wake.notify_one();
        return CSPD_OK;
    });
}

cspd_status cspd_serve_poll(cspd_server_t s, uint64_t job_id, int64_t timeout_us, cspd_job_stats *stats)
{
    return guarded([&]() -> cspd_status {
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
    });
}

void cspd_serve_destroy(cspd_server_t s)
{
    try {
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
    } catch (...) {
        // nothing may cross the C ABI; the object is left as it is
    }
}

}  // extern "C"
