// trace.cpp -- optional per-kernel timing (process-wide).
//
// When enabled, every kernel launch of the library is bracketed by two HIP events on its
// own stream; superdc_kernel_times() waits for the recorded events and returns the summed
// durations and launch counts per kernel, then starts a new collection.  The device work
// counters of some kernels (atomic adds at the end of each wavefront) can be switched on
// with the events or on their own, so that a timed pass need not pay for them.  Off by default;
// not for use while a stream is being captured into a graph.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "common.h"

namespace sdc {
namespace {

struct Mark {
    int kid;
    hipEvent_t e0, e1;
};

struct Tracer {
    std::mutex mu;
    bool events = false;    // HIP events around every launch
    bool counters = false;  // device work counters of the kernels that have them
    unsigned long long *work = nullptr;  // [KID_COUNT][TRACE_WORDS] device counters
                                         // (device `work_dev`)
    int work_dev = -1;
    std::vector<hipEvent_t> pool;  // idle events
    std::vector<Mark> marks;       // recorded, not yet collected
};

Tracer &tracer() {
    static Tracer t;
    return t;
}

hipEvent_t take(Tracer &t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

const char *kNames[KID_COUNT] = {
    "k_validate", "k_fmm_boxes", "k_fmm_lists", "k_secular", "k_secular_fmm", "k_pack_ke",
    "k_loewner", "k_bnorm", "k_apply_mfma", "k_apply_valu", "k_bwd", "k_bwd_rho",
    "k_leaf_jacobi", "k_merge", "k_assemble", "k_permute", "k_leaf_apply", "k_status_or",
    "k_fill", "k_leaf_vectors", "k_fmmv_pack", "k_fmmv_sources", "k_fmmv_eval",
    "k_fmmv_eval_mfma", "k_fmml_pack", "k_fmml_moments", "k_loewner_fmm", "k_deflate",
    "k_defl_place", "k_defl_rotate", "k_copy_rows", "k_fmm_local", "k_divide", "k_sort_pass"};

}  // namespace

unsigned long long *trace_work(int kid) {
    Tracer &t = tracer();
    if (!t.counters) return nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != t.work_dev || !t.work) return nullptr;
    return t.work + (size_t)kid * TRACE_WORDS;
}

TraceScope::TraceScope(int kid, hipStream_t s) : kid_(kid), s_(s) {
    Tracer &t = tracer();
    if (!t.events) return;  // racy read is fine: enabling is not synchronised with launches
    std::lock_guard<std::mutex> g(t.mu);
    e0_ = take(t);
    e1_ = take(t);
    if (e0_ && e1_) (void)hipEventRecord(e0_, s_);
}

TraceScope::~TraceScope() {
    if (!e0_ || !e1_) return;
    Tracer &t = tracer();
    std::lock_guard<std::mutex> g(t.mu);
    (void)hipEventRecord(e1_, s_);
    t.marks.push_back(Mark{kid_, e0_, e1_});
}

}  // namespace sdc

using namespace sdc;

extern "C" {

int superdc_kernel_timing(int enable) {
    if (enable < 0 || enable > 3) return SUPERDC_EINVAL;
    Tracer &t = tracer();
    std::lock_guard<std::mutex> g(t.mu);
    if (enable == 1 || enable == 3) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return SUPERDC_EHIP;
        if (t.work && t.work_dev != dev) {
            (void)hipFree(t.work);
            t.work = nullptr;
        }
        const size_t bytes = sizeof(unsigned long long) * KID_COUNT * TRACE_WORDS;
        if (!t.work) {
            if (hipMalloc(&t.work, bytes) != hipSuccess) {
                t.work = nullptr;
                return SUPERDC_ENOMEM;
            }
            t.work_dev = dev;
        }
        if (hipMemset(t.work, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return SUPERDC_EHIP;
    }
    t.events = enable == 1 || enable == 2;
    t.counters = enable == 1 || enable == 3;
    return SUPERDC_OK;
}

// copy the counters to the host and clear them
static int collect(Tracer &t, unsigned long long (&h)[KID_COUNT * TRACE_WORDS]) {
    if (t.work) {
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(h, t.work, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemset(t.work, 0, sizeof(h)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return SUPERDC_EHIP;
    }
    return SUPERDC_OK;
}

int superdc_kernel_work(double *pairs, int32_t count) {
    if (count < 0 || (count > 0 && !pairs)) return SUPERDC_EINVAL;
    Tracer &t = tracer();
    std::lock_guard<std::mutex> g(t.mu);
    unsigned long long h[KID_COUNT * TRACE_WORDS] = {0};
    if (collect(t, h) != SUPERDC_OK) return SUPERDC_EHIP;
    for (int i = 0; i < count; ++i) pairs[i] = i < KID_COUNT ? (double)h[i * TRACE_WORDS] : 0.0;
    return KID_COUNT;
}

int superdc_kernel_counters(double *out, int32_t count) {
    if (count < 0 || (count > 0 && !out)) return SUPERDC_EINVAL;
    Tracer &t = tracer();
    std::lock_guard<std::mutex> g(t.mu);
    unsigned long long h[KID_COUNT * TRACE_WORDS] = {0};
    if (collect(t, h) != SUPERDC_OK) return SUPERDC_EHIP;
    for (int i = 0; i < count; ++i)
        for (int w = 0; w < TRACE_WORDS; ++w)
            out[i * TRACE_WORDS + w] = i < KID_COUNT ? (double)h[i * TRACE_WORDS + w] : 0.0;
    return KID_COUNT;
}

int superdc_kernel_times(double *ms, int32_t *launches, int32_t count) {
    if (count < 0 || (count > 0 && (!ms || !launches))) return SUPERDC_EINVAL;
    if (count == 0) return KID_COUNT;  // size query: collects nothing
    Tracer &t = tracer();
    std::vector<Mark> marks;
    {
        std::lock_guard<std::mutex> g(t.mu);
        marks.swap(t.marks);
    }
    for (int i = 0; i < count; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    int rc = SUPERDC_OK;
    for (const Mark &m : marks) {
        float dt = 0.f;
        if (hipEventSynchronize(m.e1) != hipSuccess ||
            hipEventElapsedTime(&dt, m.e0, m.e1) != hipSuccess)
            rc = SUPERDC_EHIP;
        if (m.kid < count) {
            ms[m.kid] += dt;
            launches[m.kid] += 1;
        }
    }
    std::lock_guard<std::mutex> g(t.mu);
    for (const Mark &m : marks) {
        t.pool.push_back(m.e0);
        t.pool.push_back(m.e1);
    }
    return rc == SUPERDC_OK ? KID_COUNT : rc;
}

const char *superdc_kernel_name(int32_t id) {
    return id >= 0 && id < KID_COUNT ? kNames[id] : "unknown";
}

}  // extern "C"
