// Opt-in per-kernel timing of the library's own launches: when enabled, every
// launch is bracketed by two HIP events on its stream; cvr_profile_read waits
// for the recorded events and returns the summed durations per kernel kind.
#include "cvr_internal.h"

#include <mutex>

namespace cvr {

namespace {
struct Pair {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pair> g_pending;
std::vector<hipEvent_t> g_pool;
double g_ms[kProfKinds] = {};
int64_t g_count[kProfKinds] = {};

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain_locked()
{
    for (Pair& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_ms[p.kind] += ms;
            g_count[p.kind] += 1;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}
}  // namespace

ProfScope::ProfScope(int kind, hipStream_t s) : kind_(kind), s_(s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    a_ = take_event();
    if (a_) (void)hipEventRecord(static_cast<hipEvent_t>(a_), s_);
}

ProfScope::~ProfScope()
{
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (!b) {
        g_pool.push_back(static_cast<hipEvent_t>(a_));
        return;
    }
    (void)hipEventRecord(b, s_);
    g_pending.push_back(Pair{kind_, static_cast<hipEvent_t>(a_), b});
    if (g_pending.size() > 100000) drain_locked();
}

}  // namespace cvr

using namespace cvr;

extern "C" cvr_status cvr_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return CVR_OK;
}

extern "C" cvr_status cvr_profile_read(int32_t kind, double* total_ms, int64_t* launches, int32_t reset)
{
    if (kind < 0 || kind >= kProfKinds) return fail(CVR_EINVAL, "cvr_profile_read: bad kind");
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    if (total_ms) *total_ms = g_ms[kind];
    if (launches) *launches = g_count[kind];
    if (reset) {
        g_ms[kind] = 0.0;
        g_count[kind] = 0;
    }
    return CVR_OK;
}
