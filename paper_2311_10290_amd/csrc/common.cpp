// Library-wide host helpers: thread-local error text, per-kernel event
// timing, growable device buffers.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lap_host.h"

namespace lap {

static thread_local std::string t_err;

int fail(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

namespace {
struct ProfEntry {
    double ms = 0.0;
    int64_t launches = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, ProfEntry> g_prof;
const char *kKernelNames[] = {"wilson_wave", "wilson_lane",    "wilson_group", "wilson_lds", "spantree",
                              "loop_included", "pair_paths", "pair_assemble", "lv_rows", "absorbed",
                              "assemble",    "batch",         "batch_assemble"};
}  // namespace

Timer::Timer() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    on = g_prof_on;
}

void Timer::begin(const char *name, hipStream_t s) {
    if (!on) return;
    PendingEvent p;
    p.name = name;
    if (hipEventCreate(&p.a) != hipSuccess) return;
    if (hipEventCreate(&p.b) != hipSuccess) {
        (void)hipEventDestroy(p.a);
        return;
    }
    (void)hipEventRecord(p.a, s);
    pending.push_back(p);
}

void Timer::end(hipStream_t s) {
    if (!on || pending.empty()) return;
    (void)hipEventRecord(pending.back().b, s);
}

void Timer::collect() {
    if (!on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &p : pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_prof[p.name].ms += ms;
            g_prof[p.name].launches += 1;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    pending.clear();
}

Timer::~Timer() {
    for (auto &p : pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
}

int DevBuf::ensure(size_t want) {
    if (want <= bytes && ptr) return LAP_OK;
    release();
    if (want == 0) want = 8;
    if (hipMalloc(&ptr, want) != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        return LAP_ENOMEM;
    }
    bytes = want;
    return LAP_OK;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

}  // namespace lap

using namespace lap;

extern "C" const char *lap_last_error(void) { return t_err.c_str(); }

extern "C" int lap_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return LAP_OK;
}

extern "C" int lap_prof_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.clear();
    return LAP_OK;
}

extern "C" int lap_prof_read(const char *kernel, double *total_ms, int64_t *launches) {
    if (!kernel) return fail(LAP_EINVAL, "kernel name is NULL");
    bool known = false;
    for (const char *k : kKernelNames) known |= std::strcmp(k, kernel) == 0;
    if (!known) return fail(LAP_EINVAL, std::string("unknown kernel name ") + kernel);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    auto it = g_prof.find(kernel);
    if (total_ms) *total_ms = it == g_prof.end() ? 0.0 : it->second.ms;
    if (launches) *launches = it == g_prof.end() ? 0 : it->second.launches;
    return LAP_OK;
}
