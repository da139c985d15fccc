// Host-side context of libnbreg (internal; the public ABI is include/nbreg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "nbreg.h"
#include "nb_internal.h"

enum {
    NB_CLASS_FORCE = 0,
    NB_CLASS_MERGE = 1,
    NB_CLASS_PREDICT = 2,
    NB_CLASS_ADJOINT = 3,
    NB_CLASS_BATCHED = 4,
    NB_CLASS_REDO = 5,
    NB_CLASS_STEP = 6,
    NB_CLASS_SCHED = 7,
    NB_CLASS_RADIUS = 8,
    NB_NCLASS = 9
};

namespace nbrt {
// Batched ensemble: a kernel shape (index into nb::kBatchedShape) and the
// work cap (items per CU).
struct BatchedChoice {
    int shape;
    int items_per_cu;
};
struct PendingTiming {
    int cls;
    hipEvent_t start, stop;
};
struct BatchedCache;   // defined in nb_batched.hip
void batched_release(nb_ctx *ctx);
}  // namespace nbrt

struct nb_ctx {
    int device = -1;
    bool usable = false;   // false: host-only context (argument checks only)
    int cu_count = 0;
    hipStream_t stream = nullptr;
    hipError_t last_hip_error = hipSuccess;
    // scratch
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    size_t scratch_limit = 0;
    // second buffer for entry points that call other entry points (which
    // use 'scratch') while holding data of their own
    void *aux = nullptr;
    size_t aux_bytes = 0;
    // plan control
    nb::Plan forced{};
    bool has_forced = false;
    char last_plan[256] = "none";
    std::map<std::tuple<int, int64_t, int64_t>, nb::Plan> tuned;
    // mixed precision: target relative error per row and safety factor of
    // the rounding-error estimate that triggers an FP64 recompute (tol 0: off)
    double mixed_tol = 5e-6;
    double mixed_safety = 32.0;
    int32_t redo_rows_limit = 0;   // refined rows with buffered partials (0: automatic)
    // timing
    bool timing = false;
    std::vector<nbrt::PendingTiming> pending;
    std::vector<hipEvent_t> free_events;
    double ms[NB_NCLASS] = {};
    int64_t launches[NB_NCLASS] = {};
    // device words owned by the context for its whole life (never reallocated):
    // [0] the refinement counter of nb_regular_force
    int32_t *words = nullptr;
    // device address of the library's fixed workspace on this context's
    // device (nb_regular_force_noalloc); shared by every context on the device
    void *fixed_scratch = nullptr;
    int32_t *last_redo_counter = nullptr;   // device counter of the last mixed call
    // batched entry point: cached device metadata and graphs per shape
    std::vector<nbrt::BatchedCache *> batched;
    // batched kernel shape: forced (tests, the tuner) or tuned per ensemble
    bool has_batched_forced = false;
    nbrt::BatchedChoice batched_forced{0, 64};
    std::map<uint64_t, nbrt::BatchedChoice> batched_tuned;
};

namespace nbrt {
int hip_fail(nb_ctx *ctx, hipError_t e);
int ensure_scratch(nb_ctx *ctx, size_t bytes);
int ensure_aux(nb_ctx *ctx, size_t bytes);
hipError_t timed_begin(nb_ctx *ctx, int cls, hipEvent_t *ev);
hipError_t timed_end(nb_ctx *ctx, int cls, hipEvent_t *ev);
int64_t bucket_log2(int64_t v);
double redo_k(const nb_ctx *ctx);
nb::Plan auto_plan(const nb_ctx *ctx, int64_t n, int32_t n_i, bool mixed);
int64_t max_splits(int64_t n, int mapping);
int64_t default_splits(const nb_ctx *ctx, int64_t n, int32_t n_i, int mapping, int rows);
void finish_plan(nb::Plan &p, int64_t n, int32_t n_i, int64_t *split_len);
}  // namespace nbrt
