// Device arenas of the batched counter and its launch sequence.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm.h"

namespace pm {

struct Prog;
struct Job;

// Per-batch device buffers, sized for `cap` variants and `bitmap_words`
// words of footprint bitmap.  Owned by a pm_ctx.
struct Arena {
    size_t cap = 0;
    size_t bitmap_words = 0;
    Prog *prog = nullptr;        // [cap]
    Job *jobs = nullptr;         // [cap * MAXJOB]
    int64_t *varwords = nullptr; // [cap]
    int64_t *varoff = nullptr;   // [cap]
    int64_t *varchunks = nullptr; // [cap]: chunks, then their inclusive prefix
    int64_t *varsegs = nullptr;   // [cap]: fill segments, then their inclusive prefix
    int64_t *jobres = nullptr;   // [cap * MAXJOB]
    int64_t *foot = nullptr;     // [cap * MAXARR * 2]
    int64_t *meta = nullptr;     // [8]: chunks, words used, fill segments, ticket, words requested
    uint64_t *bitmap = nullptr;  // [bitmap_words]
};

size_t arena_bytes_per_variant();

// Enqueue the six counter launches for nv variants already in device
// memory (d_var) on stream s.  d_counts / model / d_pred may be null.
// ev: null, or 7 events recorded around the six launches.
int launch_batch(const Arena &ar, int nv, const pm_variant *d_var,
                 pm_counts *d_counts, const pm_model *model, double *d_pred,
                 int32_t *d_status, hipStream_t s, int n_cu,
                 hipEvent_t *ev = nullptr);

// Host execution of the same per-variant code (descriptor, jobs, items,
// fill, finalize), one variant at a time; for unit tests on machines
// without a GPU.  `sequential`: the one-pass expansion instead of the
// per-statement one.  Returns a pm_status.
int count_host(const pm_variant &v, pm_counts *out, int64_t *foot_out, bool sequential);

}  // namespace pm
