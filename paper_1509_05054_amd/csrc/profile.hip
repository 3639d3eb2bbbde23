// Optional per-kernel timing for measurement tools (dl_profile_enable /
// dl_profile_read): each launch is bracketed by two HIP events recorded on the
// launch's own stream.  Host-side bookkeeping only; off by default.
#include <vector>

#include "dl_internal.h"

namespace dlk {
namespace {

struct Rec {
    int kernel;
    hipEvent_t start, stop;
};

bool g_on = false;
int g_cap = 0;
std::vector<Rec> g_recs;          // recorded launches, in order
std::vector<hipEvent_t> g_pool;   // events available for reuse
int g_open = -1;                  // index of the launch between begin and end

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

void release_all()
{
    for (Rec &r : g_recs) {
        if (r.start)
            g_pool.push_back(r.start);
        if (r.stop)
            g_pool.push_back(r.stop);
    }
    g_recs.clear();
    g_open = -1;
}

}  // namespace

void prof_begin(int kernel, hipStream_t st)
{
    if (!g_on || (int)g_recs.size() >= g_cap)
        return;
    Rec r{kernel, take_event(), nullptr};
    if (!r.start)
        return;
    if (hipEventRecord(r.start, st) != hipSuccess) {
        g_pool.push_back(r.start);
        return;
    }
    g_recs.push_back(r);
    g_open = (int)g_recs.size() - 1;
}

void prof_end(int kernel, hipStream_t st)
{
    if (!g_on || g_open < 0)
        return;
    Rec &r = g_recs[g_open];
    g_open = -1;
    if (r.kernel != kernel)
        return;
    r.stop = take_event();
    if (r.stop && hipEventRecord(r.stop, st) != hipSuccess) {
        g_pool.push_back(r.stop);
        r.stop = nullptr;
    }
}

}  // namespace dlk

extern "C" {

dl_status dl_profile_enable(int on, int max_launches)
{
    if (on && max_launches < 1)
        return DL_EINVAL;
    dlk::release_all();
    dlk::g_on = on != 0;
    dlk::g_cap = on ? max_launches : 0;
    if (!on) {
        for (hipEvent_t e : dlk::g_pool)
            (void)hipEventDestroy(e);
        dlk::g_pool.clear();
    }
    return DL_OK;
}

dl_status dl_profile_read(double *ms, long long *launches, int count)
{
    if (!ms || !launches || count < 0 || count > DL_K_COUNT)
        return DL_EINVAL;
    dl_status rc = DL_OK;
    for (const dlk::Rec &r : dlk::g_recs) {
        if (!r.stop)
            continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) {
            rc = DL_EHIP;
            continue;
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) {
            rc = DL_EHIP;
            continue;
        }
        if (r.kernel >= 0 && r.kernel < count) {
            ms[r.kernel] += t;
            launches[r.kernel] += 1;
        }
    }
    dlk::release_all();
    return rc;
}

}  // extern "C"
