// Per-launch kernel timing with HIP events (cspd_profile_*).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cspd_internal.h"

namespace cspd {

struct ProfileToken {
    int entry;
    hipEvent_t start;
    hipEvent_t stop;
};

namespace {

struct Entry {
    std::string label;
    std::vector<ProfileToken *> pending;
    int64_t launches = 0;
    double total_ms = 0.0;
};

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Entry> g_entries;

int entry_for(const char *label)
{
    for (size_t i = 0; i < g_entries.size(); ++i)
        if (g_entries[i].label == label) return (int)i;
    g_entries.push_back(Entry{label, {}, 0, 0.0});
    return (int)g_entries.size() - 1;
}

void settle_locked()
{
    for (Entry &e : g_entries) {
        for (ProfileToken *t : e.pending) {
            float ms = 0.0f;
            if (hipEventSynchronize(t->stop) == hipSuccess &&
                hipEventElapsedTime(&ms, t->start, t->stop) == hipSuccess) {
                e.total_ms += ms;
                e.launches += 1;
            }
            (void)hipEventDestroy(t->start);
            (void)hipEventDestroy(t->stop);
            delete t;
        }
        e.pending.clear();
    }
}

}  // namespace

namespace {
thread_local int t_suspended = 0;   // launches being captured into a graph record no events
}

ProfileSuspend::ProfileSuspend() { ++t_suspended; }
ProfileSuspend::~ProfileSuspend() { --t_suspended; }

ProfileToken *profile_begin(const char *label, hipStream_t stream)
{
    if (!g_on.load(std::memory_order_relaxed) || t_suspended) return nullptr;
    ProfileToken *t = new ProfileToken();
    // timing-only events: no system-scope fence (cache writeback and
    // invalidation) at each record, which would slow the kernels that follow
    constexpr unsigned kFlags = hipEventDisableSystemFence;
    if (hipEventCreateWithFlags(&t->start, kFlags) != hipSuccess) { delete t; return nullptr; }
    if (hipEventCreateWithFlags(&t->stop, kFlags) != hipSuccess) {
        (void)hipEventDestroy(t->start);
        delete t;
        return nullptr;
    }
    {
        std::lock_guard<std::mutex> g(g_mu);
        t->entry = entry_for(label);
    }
    (void)hipEventRecord(t->start, stream);
    return t;
}

void profile_end(ProfileToken *t, hipStream_t stream)
{
    if (!t) return;
    (void)hipEventRecord(t->stop, stream);
    std::lock_guard<std::mutex> g(g_mu);
    g_entries[t->entry].pending.push_back(t);
}

ProfileToken *profile_open(const char *label, hipEvent_t *start, hipEvent_t *stop)
{
    *start = nullptr;
    *stop = nullptr;
    if (!g_on.load(std::memory_order_relaxed) || t_suspended) return nullptr;
    ProfileToken *t = new ProfileToken();
    constexpr unsigned kFlags = hipEventDisableSystemFence;
    if (hipEventCreateWithFlags(&t->start, kFlags) != hipSuccess) { delete t; return nullptr; }
    if (hipEventCreateWithFlags(&t->stop, kFlags) != hipSuccess) {
        (void)hipEventDestroy(t->start);
        delete t;
        return nullptr;
    }
    {
        std::lock_guard<std::mutex> g(g_mu);
        t->entry = entry_for(label);
    }
    *start = t->start;
    *stop = t->stop;
    return t;
}

void profile_close(ProfileToken *t)
{
    if (!t) return;
    std::lock_guard<std::mutex> g(g_mu);
    g_entries[t->entry].pending.push_back(t);
}

}  // namespace cspd

using namespace cspd;

extern "C" {

cspd_status cspd_profile_enable(int32_t on)
{
    return guarded([&]() -> cspd_status {
        g_on.store(on ? 1 : 0);
        return CSPD_OK;
    });
}

int32_t cspd_profile_read(int32_t idx, char *name, int32_t name_len, int64_t *launches, double *total_ms)
{
    try {
        std::lock_guard<std::mutex> g(g_mu);
        settle_locked();
        const int32_t n = (int32_t)g_entries.size();
        if (idx < 0 || idx >= n) return n;
        const Entry &e = g_entries[idx];
        if (name && name_len > 0) {
            std::strncpy(name, e.label.c_str(), (size_t)name_len - 1);
            name[name_len - 1] = 0;
        }
        if (launches) *launches = e.launches;
        if (total_ms) *total_ms = e.total_ms;
        return n;
    } catch (...) {
        return CSPD_E_DEVICE;
    }
}

void cspd_profile_reset(void)
{
    try {
        std::lock_guard<std::mutex> g(g_mu);
        settle_locked();
        g_entries.clear();
    } catch (...) {
        // nothing may cross the C ABI; the object is left as it is
    }
}

}  // extern "C"
