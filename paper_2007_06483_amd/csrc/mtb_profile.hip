// mtb_profile.hip -- optional per-kernel timing with HIP events.
//
// While a thread has profiling switched on (mtb_profile_begin), every kernel
// the library launches from that thread carries a start and a stop event in
// its own dispatch (hipExtLaunchKernel), so no marker is queued between
// kernels; mtb_profile_end waits for them and reports the total time per
// kernel name.  Switched off (the default), a launch costs one thread-local
// flag test.

#include <string.h>

#include <vector>

#include "mtb_internal.h"

namespace mtb {
namespace {

struct Record {
    const char *name;
    hipEvent_t start, stop;
};

thread_local bool t_enabled = false;
thread_local bool t_paused = false;
thread_local char t_filter[48] = {0};  // empty: every kernel
thread_local std::vector<Record> t_records;
thread_local hipError_t t_error = hipSuccess;

// Events are reused across profiling sessions: creating one per launch costs
// enough host time to starve the GPU between short kernels.  Kept per device.
struct PooledEvent {
    int device;
    hipEvent_t event;
};
thread_local std::vector<PooledEvent> t_pool;

hipEvent_t take_event(hipError_t *err)
{
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess)
        return nullptr;
    for (size_t i = t_pool.size(); i-- > 0;) {
        if (t_pool[i].device == dev) {
            hipEvent_t e = t_pool[i].event;
            t_pool.erase(t_pool.begin() + i);
            return e;
        }
    }
    hipEvent_t e = nullptr;
    // Timing only: no system-scope fence (cache writeback) when the event completes.
    *err = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return *err == hipSuccess ? e : nullptr;
}

void give_event(hipEvent_t e)
{
    int dev = 0;
    if (e && hipGetDevice(&dev) == hipSuccess)
        t_pool.push_back(PooledEvent{dev, e});
}

}  // namespace

ProfEvents prof_take(const char *name)
{
    ProfEvents ev;
    if (!t_enabled || t_paused || (t_filter[0] && strcmp(t_filter, name) != 0))
        return ev;
    hipError_t r = hipSuccess;
    ev.start = take_event(&r);
    if (r == hipSuccess)
        ev.stop = take_event(&r);
    if (r != hipSuccess) {
        t_error = r;
        give_event(ev.start);
        give_event(ev.stop);
        return ProfEvents();
    }
    return ev;
}

void prof_commit(const char *name, const ProfEvents &ev, hipError_t launched)
{
    if (!ev.start)
        return;
    if (launched != hipSuccess) {
        give_event(ev.start);
        give_event(ev.stop);
        return;
    }
    t_records.push_back(Record{name, ev.start, ev.stop});
}

}  // namespace mtb

using namespace mtb;

extern "C" {

mtb_status mtb_profile_begin(const char *kernel_name)
{
    if (t_enabled || (kernel_name && strlen(kernel_name) >= sizeof(t_filter)))
        return MTB_ERR_INVALID_ARG;
    t_filter[0] = 0;
    if (kernel_name)
        strcpy(t_filter, kernel_name);
    t_records.clear();
    t_error = hipSuccess;
    t_enabled = true;
    t_paused = false;
    return MTB_OK;
}

mtb_status mtb_profile_pause(int32_t paused)
{
    if (!t_enabled)
        return MTB_ERR_INVALID_ARG;
    t_paused = paused != 0;
    return MTB_OK;
}

mtb_status mtb_profile_end(mtb_kernel_time *h_out, int32_t capacity, int32_t *h_count)
{
    if (!t_enabled)
        return MTB_ERR_INVALID_ARG;
    t_enabled = false;
    t_paused = false;
    mtb_status status = t_error == hipSuccess ? MTB_OK : MTB_ERR_DEVICE;
    int32_t count = 0;
    for (const Record &r : t_records) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            status = MTB_ERR_DEVICE;
        give_event(r.start);
        give_event(r.stop);
        int32_t i = 0;
        while (i < count && strcmp(h_out[i].name, r.name) != 0)
            ++i;
        if (i == count) {
            if (!h_out || count >= capacity) {
                status = status == MTB_OK ? MTB_ERR_WORKSPACE : status;
                continue;
            }
            memset(&h_out[i], 0, sizeof(h_out[i]));
            strncpy(h_out[i].name, r.name, sizeof(h_out[i].name) - 1);
            ++count;
        }
        h_out[i].launches += 1;
        h_out[i].total_ms += ms;
    }
    t_records.clear();
    if (h_count)
        *h_count = count;
    return status;
}

}  // extern "C"
