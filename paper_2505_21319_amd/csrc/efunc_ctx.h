// Host-side internals shared by the C-ABI translation units: the context
// object behind efunc_ctx and the error reporting helpers.  Not part of the
// public interface (include/efunc.h is).
#pragma once

#include "efunc.h"
#include "efunc_internal.h"

#include <vector>

struct efunc_ctx {
    efunc_config cfg;
    efunc::Layout layout;
    efunc::Geo geo;
    efunc::Work w;
    hipStream_t last_stream;
    int device;
    std::vector<void*> allocs;
    int64_t alloc_bytes = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;  // 2 * MAX_TIMED when timing has been enabled
    int nrec = 0;
};

namespace efunc {

constexpr int MAX_TIMED = 4096;

// Set the thread-local error message and return code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);
void clear_error();
// Check a tuning record against the limits of the workspace.
int check_tuning(const efunc_tuning* t);
// Channel layout of a model variant; returns EFUNC_OK or EFUNC_EINVAL (message set).
int make_layout(const efunc_config* cfg, Layout* out);

}  // namespace efunc
