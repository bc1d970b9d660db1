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
//
// Variants handed on by the expansion kernels claim their bitmap words and
// their places in three work lists with atomics: every count or footprint
// chunk, every fill segment and every variant left to finish.  A list
// entry and its running chunk (segment) offset come from one 64-bit atomic
// (entry number in the bits from LIST_POS up, offset below), so offsets
// grow with the entry number and a chunk finds its entry by binary search.
constexpr int LIST_POS = 47;
constexpr int64_t LIST_OFF_MASK = (1ll << LIST_POS) - 1;
constexpr int64_t MAX_VARIANT_CHUNKS = 1ll << 30;  // 2^30 * 2048 outer points
// Internal status of a variant the expansion kernel handed on to the
// chip-wide kernels (they replace it with the variant's final status).
constexpr int PM_DEFER = 1;
// meta holds two halves of META_WORDS: a batch uses half `parity` and its
// expansion kernel clears the other for the next batch.
constexpr int META_WORDS = 8;
enum {
    M_CHUNKS = 0,  // packed: count-list entries, chunks
    M_WORDS = 1,   // bitmap words claimed (requested)
    M_SEGS = 2,    // packed: fill-list entries, segments
    M_DEFER = 3,   // variants handed on
    M_USED = 4,    // end of the last bitmap that fitted
    M_TICKET = 5,  // chip-wide kernel: work items taken
    M_ZDONE = 6,   // chip-wide kernel: bitmap clearing items done
};
struct Arena {
    size_t cap = 0;
    size_t bitmap_words = 0;
    int parity = 0;               // meta half of the next batch
    Prog *prog = nullptr;         // [cap]
    Job *jobs = nullptr;          // [cap * MAXJOB]
    int64_t *varoff = nullptr;    // [cap]: bitmap word offset of each variant
    int32_t *clist = nullptr;     // [cap]: variants with chunks, in claim order
    int64_t *cend = nullptr;      // [cap]: their inclusive chunk prefix
    int32_t *slist = nullptr;     // [cap]: variants with fill segments
    int64_t *send = nullptr;      // [cap]: their inclusive segment prefix
    int32_t *dlist = nullptr;     // [cap]: variants left to finish
    int64_t *jobres = nullptr;    // [cap * MAXJOB]
    int64_t *foot = nullptr;      // [cap * MAXARR * 2]
    int64_t *vdone = nullptr;     // [cap * 2]: chunks and fill segments done
    int64_t *meta = nullptr;      // [2 * META_WORDS]
    uint64_t *bitmap = nullptr;   // [bitmap_words]
};

size_t arena_bytes_per_variant();

// Enqueue the counter launches for nv variants already in device memory
// (d_var) on stream s; flips ar.parity.  d_counts / model / d_pred may be
// null.  ev: null, or events recorded around the three phases (the
// expansion kernel, the gap between the kernels, the chip-wide kernel);
// the first `nmark` of the four are recorded (2: around the expansion
// kernel only).
// Schedule of the batched counter (pm_schedule): the most items a
// variant's count jobs may hold to be counted by the work-group that
// expands it (k_build; k_fused), and the work-groups per CU of the
// chip-wide kernels.
struct Sched {
    int64_t inblock_items = 4096;
    int64_t fused_items = 1 << 20;
    int tail_wgs_per_cu = 4;
};

int launch_batch(Arena &ar, const Sched &sc, int nv, const pm_variant *d_var,
                 pm_counts *d_counts, const pm_model *model, double *d_pred,
                 int32_t *d_status, hipStream_t s, int n_cu,
                 hipEvent_t *ev = nullptr, int nmark = 4);
// The same in two parts: the expansion kernel (events 0 and 1; flips
// ar.parity) and the chip-wide kernel for the variants it handed on
// (events 2 and 3), which a caller that has read the expansion's meta half may
// skip when it handed none on.
int launch_expand(Arena &ar, const Sched &sc, int nv, const pm_variant *d_var, pm_counts *d_counts,
                  const pm_model *model, double *d_pred, int32_t *d_status, hipStream_t s,
                  hipEvent_t *ev, int nmark);
int launch_rest(Arena &ar, const Sched &sc, int nv, pm_counts *d_counts, const pm_model *model,
                double *d_pred, int32_t *d_status, hipStream_t s, int n_cu, hipEvent_t *ev,
                int nmark);

// Host execution of the same per-variant code (descriptor, jobs, items,
// fill, finalize), one variant at a time; for unit tests on machines
// without a GPU.  `sequential`: the one-pass expansion instead of the
// per-statement one.  Returns a pm_status.
int count_host(const pm_variant &v, pm_counts *out, int64_t *foot_out, bool sequential);

}  // namespace pm
