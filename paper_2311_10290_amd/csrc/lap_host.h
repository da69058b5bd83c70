// Host-side internals of the library: graph handle, workspace, ingest.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lap.h"

namespace lap {

struct HostCSR {
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<int32_t> old_ids;
};

int build_host_csr(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst, bool keep_lcc,
                   HostCSR &out, std::string &err);

// Set the thread's error text and return code.
int fail(int code, const std::string &msg);

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::lap::fail(e_ == hipErrorOutOfMemory ? LAP_ENOMEM : LAP_EDEVICE,     \
                               std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

// Optional per-kernel timing: events around launches, accumulated by name
// after the caller's streams have been synchronised (lap_prof_*).
struct Timer {
    struct PendingEvent {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<PendingEvent> pending;
    bool on = false;
    Timer();
    ~Timer();
    void begin(const char *name, hipStream_t s);
    void end(hipStream_t s);
    void collect();
};

// A device allocation that only grows.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t want);
    void release();
    template <class T>
    T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace lap
