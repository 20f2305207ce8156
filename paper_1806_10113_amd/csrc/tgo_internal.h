// Internal host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/tgo.h"
#include "model_dev.h"

namespace tgo {

// Thread-local error detail behind tgo_last_error().
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define TGO_HIP(call)                                      \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return ::tgo::hip_fail(e_, #call); \
    } while (0)

// Validate a model and derive the kernel constants.
int make_rates(const tgo_model *m, Rates *r);

// Device workspace owned by the library, one per (device, stream), grown on
// demand (a growth waits for the stream's earlier work) and kept until the
// process ends.  Calls on different streams get different buffers, so they
// may overlap; calls on one stream are ordered by the stream.
int workspace(size_t bytes, void **ptr, hipStream_t st);

constexpr uint64_t factorial(int n) { return n <= 1 ? 1ull : (uint64_t)n * factorial(n - 1); }

// Device-side validity of a task table: 0 (32-bit time path), 1 (64-bit path)
// or a negative TGO_E* code.  Durations must lie in [0, 2^40) ns.
constexpr int64_t MAX_DURATION = int64_t(1) << 40;

struct Partial {
    uint64_t min_t, min_r, max_t, max_r, sum_lo, sum_hi, fp;
    int32_t status, pad;
};

int launch_exhaustive(const Rates &r, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                      tgo_summary *d_out, hipStream_t st);
// Same enumeration with its scratch in a fixed per-device array (no
// allocation; the grid is bounded by the array's size).
int launch_exhaustive_noalloc(const Rates &r, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                              tgo_summary *d_out, hipStream_t st);
int launch_evaluate(const Rates &r, const tgo_task *d_tasks, int n, const uint8_t *d_orders,
                    int64_t m, int64_t *d_out, hipStream_t st);
int launch_rounds(const Rates &r, const tgo_task *d_tasks, int T, int R, int64_t *d_per_order,
                  tgo_summary *d_out, uint16_t *d_groups, hipStream_t st);
// Block partials -> summary over (T!)^R ranks of T*R tasks (T = n, R = 1 for
// one group); best / worst decoded as launch sequences.
int launch_summary_finalize(const Partial *d_parts, int nparts, int T, int R, uint64_t count, uint64_t tfact,
                            tgo_summary *d_out, hipStream_t st);
int launch_memory(const Rates &r, const tgo_task *d_tasks, const int64_t *d_mem, int n, int64_t cap,
                  int64_t *d_per_order, tgo_summary *d_out, hipStream_t st);
int launch_memory_evaluate(const Rates &r, const tgo_task *d_tasks, const int64_t *d_mem, int n, int64_t cap,
                           const uint8_t *d_orders, int64_t m, int64_t *d_out, hipStream_t st);
// Device bytes owned by a plan / a surrogate (for the server's memory budget).
size_t plan_device_bytes(const tgo_plan *p);
size_t surrogate_device_bytes(const tgo_surrogate *s);
int surrogate_reserve(tgo_surrogate *s, int max_groups, int64_t samples);
int launch_heuristic(const Rates &r, const tgo_task *d_tasks, const int32_t *d_offs, int n_groups,
                     uint8_t *d_orders, int order_stride, int64_t *d_ns, int ns_stride,
                     hipStream_t st);

}  // namespace tgo
