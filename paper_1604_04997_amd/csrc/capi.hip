// C ABI of libpm (include/pm.h): contexts, counting, prediction, fit,
// kernel launch and measurement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "counter.h"
#include "desc.h"
#include "fit.h"
#include "pm.h"
#include "pm_testing.h"
#include "suite.h"

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

const char *status_name(int s) {
    switch (s) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid descriptor or argument";
    case PM_ENOMEM: return "out of device memory / HBM budget";
    case PM_EDEVICE: return "HIP runtime error";
    case PM_ERANK: return "no non-zero feature column";
    case PM_EOVERFLOW: return "count exceeds int64";
    case PM_ETIMEDOUT: return "deadline passed";
    case PM_EBUSY: return "context busy";
    }
    return "unknown";
}

#define HIPCHK(x)                                                               \
    do {                                                                        \
        hipError_t e_ = (x);                                                    \
        if (e_ != hipSuccess)                                                   \
            return set_err(PM_EDEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

// Validation by expanding the descriptor on the host.
struct HostBuild {
    std::unique_ptr<pm::Prog> prog{new pm::Prog};
    std::unique_ptr<pm::Job[]> jobs{new pm::Job[pm::MAXJOB]};
};
thread_local HostBuild g_hb;

int validate(const pm_variant *v) {
    if (!v) return set_err(PM_EINVAL, "null variant");
    int st = pm::build_prog(*v, g_hb.prog.get(), g_hb.jobs.get());
    if (st != PM_OK)
        return set_err(st, std::string("variant of family ") + std::to_string(v->family) +
                               ": " + status_name(st));
    return PM_OK;
}

// Restores the calling thread's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

// Host-call batches up to this size get mapped-memory outputs.
constexpr int ZC_MAX = 32;

struct pm_ctx {
    int device = 0;
    size_t budget = 0;
    int n_cu = 256;
    pm::Sched sched;
    hipStream_t stream = nullptr;
    pm::Arena ar;
    size_t arena_alloc = 0;  // bytes held by ar (without bitmap)
    size_t bitmap_alloc = 0;
    // host-call staging
    pm_variant *d_var = nullptr;
    pm_counts *d_counts = nullptr;
    double *d_pred = nullptr;
    int32_t *d_status = nullptr;
    pm_variant *h_var = nullptr;
    pm_counts *h_counts = nullptr;
    double *h_pred = nullptr;
    int32_t *h_status = nullptr;
    int64_t *h_meta = nullptr;
    // outputs of small host-call batches, written by the kernels straight
    // into pinned host memory (fine-grained: visible once the kernel ends)
    pm_counts *z_counts = nullptr;
    double *z_pred = nullptr;
    int32_t *z_status = nullptr;
    pm_counts *zd_counts = nullptr;  // the same memory, device addresses
    double *zd_pred = nullptr;
    int32_t *zd_status = nullptr;
    std::vector<hipEvent_t> events;
    // Order of batches on the shared arena: a batch on another stream than
    // the previous batch's waits for an event recorded on that stream after
    // the previous batch.  The event is recorded after every batch on a
    // caller's stream; after a batch on the null stream or the context's own
    // stream (which stay valid) only when a batch on another stream needs
    // it (arena_lazy), so that batches following each other on one such
    // stream pay no event (one costs about 3 us of queue time per batch).
    hipEvent_t arena_done = nullptr;
    hipStream_t arena_stream = nullptr;
    bool arena_used = false, arena_lazy = false;
    // measurement: the last timed launch of a call that timed out (a later
    // call waits for it before reusing the events), the launch floor
    hipEvent_t measure_pending = nullptr;
    double launch_floor = 0.0;
    int profile = 0;  // 0 off, 1 every phase, 2 the expansion kernel only
    std::vector<hipEvent_t> pev;  // (PM_NPHASE + 1) per recorded batch
    int pcount = 0;
    int pevery = 1;      // events on one batch in pevery
    int64_t pseen = 0;   // batches since the window opened
    int nmarks() const { return profile == 2 ? 2 : PM_NPHASE + 1; }
    hipEvent_t *next_events() {
        if (!profile || pcount >= PM_PROFILE_MAX) return nullptr;
        if (pseen++ % pevery != 0) return nullptr;
        size_t need = (size_t)(pcount + 1) * (PM_NPHASE + 1);
        while (pev.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pev.push_back(e);
        }
        return &pev[(size_t)(pcount++) * (PM_NPHASE + 1)];
    }
};

// ------------------------------------------------ allocation-free path ---
// pm_count_device_noalloc runs the batched counter in `scratch`, a
// file-scope device array that every device the library runs on holds
// until the process ends, laid out as a counter arena (the one pm_ctx
// allocates for pm_count_device) for PM_NOALLOC_MAX_VARIANTS variants and
// PM_NOALLOC_BITMAP_BYTES of footprint bitmaps.  In host code `scratch`
// names a host-side stand-in, not the device array: its device address is
// looked up once per device (hipGetSymbolAddress, in pm_create) and only
// that address is used.
namespace noalloc {

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t CAP = PM_NOALLOC_MAX_VARIANTS;
constexpr size_t OFF_META = 0;
constexpr size_t OFF_PROG = align256(OFF_META + 16 * pm::META_WORDS);
constexpr size_t OFF_JOBS = align256(OFF_PROG + sizeof(pm::Prog) * CAP);
constexpr size_t OFF_VAROFF = align256(OFF_JOBS + sizeof(pm::Job) * CAP * pm::MAXJOB);
constexpr size_t OFF_CLIST = align256(OFF_VAROFF + 8 * CAP);
constexpr size_t OFF_CEND = align256(OFF_CLIST + 4 * CAP);
constexpr size_t OFF_SLIST = align256(OFF_CEND + 8 * CAP);
constexpr size_t OFF_SEND = align256(OFF_SLIST + 4 * CAP);
constexpr size_t OFF_DLIST = align256(OFF_SEND + 8 * CAP);
constexpr size_t OFF_JOBRES = align256(OFF_DLIST + 4 * CAP);
constexpr size_t OFF_FOOT = align256(OFF_JOBRES + 8 * CAP * pm::MAXJOB);
constexpr size_t OFF_VDONE = align256(OFF_FOOT + 16 * CAP * pm::MAXARR);
constexpr size_t OFF_BITMAP = align256(OFF_VDONE + 16 * CAP);
constexpr size_t BYTES = OFF_BITMAP + PM_NOALLOC_BITMAP_BYTES;

static __device__ __align__(256) uint8_t scratch[BYTES];

constexpr int MAX_DEVICES = 64;
struct Dev {
    uint8_t *ptr = nullptr;  // device address of `scratch` on this device
    int parity = 0;          // meta half of the next batch
};
Dev g_dev[MAX_DEVICES];
std::mutex g_mu;

__global__ void k_zero(int64_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Once per device, with that device current: the array's device address,
// and its two list-counter halves cleared (a fill kernel on `s`).
int setup(int dev, hipStream_t s) {
    if (dev < 0 || dev >= MAX_DEVICES) return set_err(PM_EDEVICE, "device number too large");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_dev[dev].ptr) return PM_OK;
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return set_err(PM_EDEVICE, "no device address for the scratch array");
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, (int64_t *)((uint8_t *)ptr + OFF_META),
                       2 * pm::META_WORDS);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    g_dev[dev].ptr = (uint8_t *)ptr;
    g_dev[dev].parity = 0;
    return PM_OK;
}

// The arena inside the array at device address `base`.
pm::Arena arena(uint8_t *base, int parity) {
    pm::Arena a;
    a.cap = CAP;
    a.bitmap_words = PM_NOALLOC_BITMAP_BYTES / 8;
    a.parity = parity;
    a.meta = (int64_t *)(base + OFF_META);
    a.prog = (pm::Prog *)(base + OFF_PROG);
    a.jobs = (pm::Job *)(base + OFF_JOBS);
    a.varoff = (int64_t *)(base + OFF_VAROFF);
    a.clist = (int32_t *)(base + OFF_CLIST);
    a.cend = (int64_t *)(base + OFF_CEND);
    a.slist = (int32_t *)(base + OFF_SLIST);
    a.send = (int64_t *)(base + OFF_SEND);
    a.dlist = (int32_t *)(base + OFF_DLIST);
    a.jobres = (int64_t *)(base + OFF_JOBRES);
    a.foot = (int64_t *)(base + OFF_FOOT);
    a.vdone = (int64_t *)(base + OFF_VDONE);
    a.bitmap = (uint64_t *)(base + OFF_BITMAP);
    return a;
}

}  // namespace noalloc

namespace {

void free_arena(pm_ctx *c) {
    pm::Arena &a = c->ar;
    (void)hipFree(a.prog);
    (void)hipFree(a.jobs);
    (void)hipFree(a.varoff);
    (void)hipFree(a.clist);
    (void)hipFree(a.cend);
    (void)hipFree(a.slist);
    (void)hipFree(a.send);
    (void)hipFree(a.dlist);
    (void)hipFree(a.jobres);
    (void)hipFree(a.foot);
    (void)hipFree(a.vdone);
    (void)hipFree(a.meta);
    (void)hipFree(c->d_var);
    (void)hipFree(c->d_counts);
    (void)hipFree(c->d_pred);
    (void)hipFree(c->d_status);
    (void)hipHostFree(c->h_var);
    (void)hipHostFree(c->h_counts);
    (void)hipHostFree(c->h_pred);
    (void)hipHostFree(c->h_status);
    uint64_t *bm = a.bitmap;
    size_t bw = a.bitmap_words;
    a = pm::Arena{};
    a.bitmap = bm;
    a.bitmap_words = bw;
    c->d_var = nullptr;
    c->d_counts = nullptr;
    c->d_pred = nullptr;
    c->d_status = nullptr;
    c->h_var = nullptr;
    c->h_counts = nullptr;
    c->h_pred = nullptr;
    c->h_status = nullptr;
    c->arena_alloc = 0;
}

int grow_cap(pm_ctx *c, size_t nv) {
    if (nv <= c->ar.cap) return PM_OK;
    size_t cap = std::max<size_t>(nv, std::min<size_t>(2 * c->ar.cap, PM_BATCH_MAX));
    cap = std::max(cap, nv);
    size_t per = pm::arena_bytes_per_variant() + sizeof(pm_variant) + sizeof(pm_counts) +
                 sizeof(double) + sizeof(int32_t);
    if (per * cap + c->bitmap_alloc > c->budget)
        return set_err(PM_ENOMEM, "batch arena exceeds the context's HBM budget");
    // batches may be in flight on caller streams: wait for the device
    (void)hipDeviceSynchronize();
    free_arena(c);
    pm::Arena &a = c->ar;
    HIPCHK(hipMalloc(&a.prog, sizeof(pm::Prog) * cap));
    HIPCHK(hipMalloc(&a.jobs, sizeof(pm::Job) * cap * pm::MAXJOB));
    HIPCHK(hipMalloc(&a.varoff, 8 * cap));
    HIPCHK(hipMalloc(&a.clist, 4 * cap));
    HIPCHK(hipMalloc(&a.cend, 8 * cap));
    HIPCHK(hipMalloc(&a.slist, 4 * cap));
    HIPCHK(hipMalloc(&a.send, 8 * cap));
    HIPCHK(hipMalloc(&a.dlist, 4 * cap));
    HIPCHK(hipMalloc(&a.jobres, 8 * cap * pm::MAXJOB));
    HIPCHK(hipMalloc(&a.foot, 16 * cap * pm::MAXARR));
    HIPCHK(hipMalloc(&a.vdone, 16 * cap));
    HIPCHK(hipMalloc(&a.meta, 16 * pm::META_WORDS));
    HIPCHK(hipMemset(a.meta, 0, 16 * pm::META_WORDS));  // both halves start clear
    HIPCHK(hipDeviceSynchronize());
    a.parity = 0;
    HIPCHK(hipMalloc(&c->d_var, sizeof(pm_variant) * cap));
    HIPCHK(hipMalloc(&c->d_counts, sizeof(pm_counts) * cap));
    HIPCHK(hipMalloc(&c->d_pred, sizeof(double) * cap));
    HIPCHK(hipMalloc(&c->d_status, sizeof(int32_t) * cap));
    HIPCHK(hipHostMalloc(&c->h_var, sizeof(pm_variant) * cap, 0));
    HIPCHK(hipHostMalloc(&c->h_counts, sizeof(pm_counts) * cap, 0));
    HIPCHK(hipHostMalloc(&c->h_pred, sizeof(double) * cap, 0));
    HIPCHK(hipHostMalloc(&c->h_status, sizeof(int32_t) * cap, 0));
    a.cap = cap;
    c->arena_alloc = per * cap;
    return PM_OK;
}

int grow_bitmap(pm_ctx *c, size_t words) {
    if (words <= c->ar.bitmap_words) return PM_OK;
    size_t w = std::max(words, c->ar.bitmap_words * 2);
    if (c->arena_alloc + w * 8 > c->budget) w = words;
    if (c->arena_alloc + w * 8 > c->budget)
        return set_err(PM_ENOMEM, "footprint bitmaps exceed the context's HBM budget");
    (void)hipDeviceSynchronize();
    (void)hipFree(c->ar.bitmap);
    c->ar.bitmap = nullptr;
    c->ar.bitmap_words = 0;
    c->bitmap_alloc = 0;
    HIPCHK(hipMalloc(&c->ar.bitmap, w * 8));
    c->ar.bitmap_words = w;
    c->bitmap_alloc = w * 8;
    return PM_OK;
}

// Make stream s wait for the previous batch on the shared arena when that
// batch ran on another stream.
int arena_enter(pm_ctx *c, hipStream_t s) {
    if (c->arena_used && c->arena_stream != s) {
        if (c->arena_lazy) HIPCHK(hipEventRecord(c->arena_done, c->arena_stream));
        HIPCHK(hipStreamWaitEvent(s, c->arena_done, 0));
    }
    return PM_OK;
}
// The batch on stream s has enqueued its last kernel.
int arena_leave(pm_ctx *c, hipStream_t s) {
    c->arena_lazy = s == nullptr || s == c->stream;
    if (!c->arena_lazy) HIPCHK(hipEventRecord(c->arena_done, s));
    c->arena_stream = s;
    c->arena_used = true;
    return PM_OK;
}

// Count (and optionally predict) nv <= cap variants from host memory.
// Batches of up to ZC_MAX variants have their outputs written by the
// kernels into mapped host memory (no device-to-host copies); larger ones
// are copied back.
int run_host_batch(pm_ctx *c, const pm_variant *v, size_t nv, pm_counts *out,
                   const pm_model *m, double *t) {
    int st = grow_cap(c, nv);
    if (st) return st;
    std::memcpy(c->h_var, v, sizeof(pm_variant) * nv);
    const bool zc = nv <= (size_t)ZC_MAX;
    pm_counts *dc = zc ? c->zd_counts : c->d_counts;
    double *dp = m ? (zc ? c->zd_pred : c->d_pred) : nullptr;
    int32_t *ds = zc ? c->zd_status : c->d_status;
    const int32_t *hs = zc ? c->z_status : c->h_status;
    // read back what the kernels wrote (copies only for large batches)
    auto fetch = [&]() -> int {
        if (!zc) {
            HIPCHK(hipMemcpyAsync(c->h_status, c->d_status, 4 * nv, hipMemcpyDeviceToHost, c->stream));
            if (out) HIPCHK(hipMemcpyAsync(c->h_counts, c->d_counts, sizeof(pm_counts) * nv, hipMemcpyDeviceToHost, c->stream));
            if (m) HIPCHK(hipMemcpyAsync(c->h_pred, c->d_pred, 8 * nv, hipMemcpyDeviceToHost, c->stream));
        }
        HIPCHK(hipStreamSynchronize(c->stream));
        return PM_OK;
    };
    // The expansion kernel finishes most variants by itself; the chip-wide
    // kernels run only when it handed some on, after the host has read the
    // statuses (one more round trip then, four launches fewer otherwise).
    hipEvent_t *ev = c->next_events();
    const int nmark = c->nmarks();
    for (int attempt = 0; attempt < 2; attempt++) {
        if ((st = arena_enter(c, c->stream))) return st;
        HIPCHK(hipMemcpyAsync(c->d_var, c->h_var, sizeof(pm_variant) * nv, hipMemcpyHostToDevice, c->stream));
        st = pm::launch_expand(c->ar, c->sched, (int)nv, c->d_var, dc, m, dp, ds, c->stream, ev,
                               nmark);
        if (st) return set_err(st, "counter launch failed");
        if ((st = arena_leave(c, c->stream))) return st;
        if ((st = fetch())) return st;
        bool nomem = false, deferred = false;
        for (size_t i = 0; i < nv; i++) {
            nomem |= hs[i] == PM_ENOMEM;
            deferred |= hs[i] == pm::PM_DEFER;
        }
        if (nomem) {  // grow the bitmap arena to what the batch asked for, expand again
            if (attempt == 1) return set_err(PM_ENOMEM, "footprint bitmaps do not fit");
            HIPCHK(hipMemcpy(c->h_meta, c->ar.meta + pm::META_WORDS * (c->ar.parity ^ 1),
                             8 * pm::META_WORDS, hipMemcpyDeviceToHost));
            st = grow_bitmap(c, (size_t)c->h_meta[pm::M_WORDS]);
            if (st) return st;
            continue;
        }
        if (deferred) {
            st = pm::launch_rest(c->ar, c->sched, (int)nv, dc, m, dp, ds, c->stream, c->n_cu, ev,
                                 nmark);
            if (st) return set_err(st, "counter launch failed");
            if ((st = arena_leave(c, c->stream))) return st;
            if ((st = fetch())) return st;
        } else if (ev) {  // phases that did not run take no time
            for (int q = 2; q < nmark; q++) (void)hipEventRecord(ev[q], c->stream);
        }
        break;
    }
    int first = PM_OK;
    for (size_t i = 0; i < nv; i++) {
        if (hs[i] != PM_OK && first == PM_OK) {
            first = hs[i];
            set_err(first, "variant " + std::to_string(i) + ": " + status_name(first));
        }
    }
    if (out) std::memcpy(out, zc ? c->z_counts : c->h_counts, sizeof(pm_counts) * nv);
    if (m && t) std::memcpy(t, zc ? c->z_pred : c->h_pred, 8 * nv);
    return first;
}

// Split into batches that fit the budget: halves on PM_ENOMEM.
int run_host(pm_ctx *c, const pm_variant *v, size_t nv, pm_counts *out,
             const pm_model *m, double *t) {
    int first = PM_OK;
    for (size_t off = 0; off < nv; off += PM_BATCH_MAX) {
        size_t nb = std::min<size_t>(PM_BATCH_MAX, nv - off);
        int st = run_host_batch(c, v + off, nb, out ? out + off : nullptr, m, t ? t + off : nullptr);
        if (st == PM_ENOMEM && nb > 1) {
            size_t h = nb / 2;
            st = run_host(c, v + off, h, out ? out + off : nullptr, m, t ? t + off : nullptr);
            int st2 = run_host(c, v + off + h, nb - h, out ? out + off + h : nullptr, m,
                               t ? t + off + h : nullptr);
            if (st == PM_OK) st = st2;
        }
        if (st != PM_OK && first == PM_OK) first = st;
    }
    return first;
}

int check_bufs(const pm_variant *v, void *const *bufs, const size_t *bytes, uint32_t nbufs) {
    size_t need[PM_MAXBUF];
    uint32_t role[PM_MAXBUF], nb = 0;
    int st = pm::buffers(*v, need, role, &nb);
    if (st) return set_err(st, "no buffer layout for this family");
    if (nbufs < nb) return set_err(PM_EINVAL, "kernel takes " + std::to_string(nb) + " buffers");
    for (uint32_t i = 0; i < nb; i++) {
        if (!bufs || !bufs[i]) return set_err(PM_EINVAL, "null buffer " + std::to_string(i));
        if (!bytes || bytes[i] < need[i])
            return set_err(PM_EINVAL, "buffer " + std::to_string(i) + " smaller than " +
                                          std::to_string(need[i]) + " bytes");
    }
    return PM_OK;
}

// Timed launches in flight at once: enough that the next launch is always
// queued behind the running one, few enough that a deadline stops the call
// soon after it passes.
constexpr int MEASURE_INFLIGHT = 4;

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Sec. 4.2 timing: `warmup` untimed launches, then `reps` launches between
// HIP events, at most MEASURE_INFLIGHT of them enqueued ahead of the last
// one that completed.  deadline_s >= 0: once that much host wall time has
// passed since the call began, nothing more is enqueued and the call
// returns PM_ETIMEDOUT; what was enqueued runs to completion on the stream
// (the next measurement on this context waits for it).
int measure_impl(pm_ctx *c, const pm_variant *v, void *const *bufs, const size_t *bytes,
                 uint32_t nbufs, void *stream, int warmup, int reps, double deadline_s,
                 double *t_reps, double *t_min, int32_t *reps_done, uint32_t *flags) {
    if (!c || !t_min || reps < 1 || warmup < 0) return set_err(PM_EINVAL, "bad argument");
    int st = validate(v);
    if (st) return st;
    st = check_bufs(v, bufs, bytes, nbufs);
    if (st) return st;
    DeviceGuard g(c->device);
    const auto t0 = std::chrono::steady_clock::now();
    auto late = [&]() { return deadline_s >= 0 && seconds_since(t0) > deadline_s; };
    hipStream_t s = (hipStream_t)stream;  // NULL: HIP's null stream
    if (c->measure_pending) {  // launches of a call that timed out
        HIPCHK(hipEventSynchronize(c->measure_pending));
        c->measure_pending = nullptr;
    }
    while ((int)c->events.size() < 2 * reps + 1) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->events.push_back(e);
    }
    *t_min = 0;
    if (reps_done) *reps_done = 0;
    if (flags) *flags = 0;
    int enq = 0, done = 0;  // timed launches enqueued, completed
    bool timed_out = false;
    // polls the end event of timed launch `done`; false on a HIP error
    auto poll = [&](hipError_t *err) -> bool {
        const hipError_t q = hipEventQuery(c->events[2 * done + 1]);
        if (q == hipSuccess) {
            done++;
            return true;
        }
        if (q != hipErrorNotReady) {
            *err = q;
            return false;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        return true;
    };
    hipError_t herr = hipSuccess;
    for (int w = 0; w < warmup && !timed_out; w++) {
        if (late()) timed_out = true;
        else if ((st = pm::launch(*v, bufs, s))) return set_err(st, "kernel launch failed");
    }
    while (enq < reps && !timed_out) {
        if (enq - done >= MEASURE_INFLIGHT) {
            if (!poll(&herr)) return set_err(PM_EDEVICE, std::string("event query: ") + hipGetErrorString(herr));
            if (late()) timed_out = true;
            continue;
        }
        if (late()) {
            timed_out = true;
            break;
        }
        HIPCHK(hipEventRecord(c->events[2 * enq], s));
        if ((st = pm::launch(*v, bufs, s))) return set_err(st, "kernel launch failed");
        HIPCHK(hipEventRecord(c->events[2 * enq + 1], s));
        enq++;
    }
    while (done < enq && !timed_out) {
        if (!poll(&herr)) return set_err(PM_EDEVICE, std::string("event query: ") + hipGetErrorString(herr));
        if (done < enq && late()) timed_out = true;
    }
    // times of the completed launches (the first `done`, in order)
    double best = 0;
    for (int r = 0; r < done; r++) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->events[2 * r], c->events[2 * r + 1]));
        const double sec = (double)ms * 1e-3;
        if (t_reps) t_reps[r] = sec;
        best = r == 0 ? sec : std::min(best, sec);
    }
    *t_min = best;
    if (reps_done) *reps_done = done;
    if (flags && done > 0 && c->launch_floor > 0 && best < 2.0 * c->launch_floor)
        *flags |= PM_MEASURE_BELOW_FLOOR;
    if (timed_out) {
        // whatever was enqueued still runs; mark its end for the next call
        HIPCHK(hipEventRecord(c->events[2 * reps], s));
        c->measure_pending = c->events[2 * reps];
        return set_err(PM_ETIMEDOUT, "measurement deadline of " + std::to_string(deadline_s) +
                                         " s passed after " + std::to_string(done) + " of " +
                                         std::to_string(reps) + " timed launches");
    }
    return PM_OK;
}

}  // namespace

extern "C" {

const char *pm_last_error(void) { return g_err.c_str(); }

pm_status pm_create(pm_ctx **out, int device, size_t budget) {
    if (!out) return (pm_status)set_err(PM_EINVAL, "null out");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return (pm_status)set_err(PM_EDEVICE, "no HIP device " + std::to_string(device));
    DeviceGuard g(device);
    auto c = std::make_unique<pm_ctx>();
    c->device = device;
    c->budget = budget ? budget : (size_t)64 << 30;
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        c->n_cu = 256;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
        return (pm_status)set_err(PM_EDEVICE, "stream creation failed");
    if (hipEventCreateWithFlags(&c->arena_done, hipEventDisableTiming) != hipSuccess)
        return (pm_status)set_err(PM_EDEVICE, "event creation failed");
    if (noalloc::setup(device, c->stream) != PM_OK) return PM_EDEVICE;
    if (hipHostMalloc(&c->h_meta, 8 * pm::META_WORDS, 0) != hipSuccess)
        return (pm_status)set_err(PM_EDEVICE, "pinned allocation failed");
    const unsigned zf = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc(&c->z_counts, sizeof(pm_counts) * ZC_MAX, zf) != hipSuccess ||
        hipHostMalloc(&c->z_pred, sizeof(double) * ZC_MAX, zf) != hipSuccess ||
        hipHostMalloc(&c->z_status, sizeof(int32_t) * ZC_MAX, zf) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->zd_counts, c->z_counts, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->zd_pred, c->z_pred, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->zd_status, c->z_status, 0) != hipSuccess)
        return (pm_status)set_err(PM_EDEVICE, "mapped pinned allocation failed");
    *out = c.release();
    return PM_OK;
}

void pm_destroy(pm_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_arena(c);
    (void)hipFree(c->ar.bitmap);
    (void)hipHostFree(c->h_meta);
    (void)hipHostFree(c->z_counts);
    (void)hipHostFree(c->z_pred);
    (void)hipHostFree(c->z_status);
    if (c->measure_pending) (void)hipEventSynchronize(c->measure_pending);
    (void)hipDeviceSynchronize();  // batches on caller streams
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    if (c->arena_done) (void)hipEventDestroy(c->arena_done);
    for (hipEvent_t e : c->pev) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->stream);
    delete c;
}

pm_status pm_count_name(int i, char *buf, size_t cap) {
    static const char *cls[pm::NCLS] = {"0", "1", "1/2", "2/2", "1/3", "2/3", "3/3", "1/4",
                                        "2/4", "3/4", "4/4", "1/>4", "2/>4", "3/>4", "4/>4"};
    static const char *kind[6] = {"add", "mul", "div", "exp", "spec", "fma"};
    static const char *sz[3] = {"4", "8", "16"};
    if (i < 0 || i >= PM_NCOUNT || !buf || cap == 0) return (pm_status)set_err(PM_EINVAL, "bad slot");
    if (i < pm::C_LDS) {
        int d = i / 45, r = i % 45;
        snprintf(buf, cap, "%s.%s.%s", d ? "gst" : "gld", sz[r / 15], cls[r % 15]);
    } else if (i < pm::C_FLOP) {
        int r = i - pm::C_LDS;
        snprintf(buf, cap, "%s.%s", r / 3 ? "lst" : "lld", sz[r % 3]);
    } else if (i < pm::C_BARWI) {
        int r = i - pm::C_FLOP;
        snprintf(buf, cap, "%s.%s", kind[r / 2], r % 2 ? "f64" : "f32");
    } else if (i < pm::C_LDSB) {
        static const char *tail[4] = {"bar.wi", "bar.wg", "wg", "wi"};
        snprintf(buf, cap, "%s", tail[i - pm::C_BARWI]);
    } else {  // LDS by bank-stride bin: broadcast, then odd, 2 x odd, ..., 32 x
        static const char *bin[pm::NLBIN] = {"b0", "b1", "b2", "b4", "b8", "b16", "b32"};
        const int r = i - pm::C_LDSB, dz = r / pm::NLBIN;
        snprintf(buf, cap, "%s.%s.%s", dz / 3 ? "lst" : "lld", sz[dz % 3], bin[r % pm::NLBIN]);
    }
    return PM_OK;
}

pm_status pm_count(pm_ctx *c, const pm_variant *v, size_t nv, pm_counts *out) {
    if (!c || (!v && nv) || (!out && nv)) return (pm_status)set_err(PM_EINVAL, "null argument");
    if (nv == 0) return PM_OK;
    DeviceGuard g(c->device);
    return (pm_status)run_host(c, v, nv, out, nullptr, nullptr);
}

pm_status pm_predict(pm_ctx *c, const pm_model *m, const pm_variant *v, size_t nv, double *t) {
    if (!c || !m || (!v && nv) || (!t && nv)) return (pm_status)set_err(PM_EINVAL, "null argument");
    if (pm::nfeat(m->proj) < 0 || (int)m->nfeat != pm::nfeat(m->proj))
        return (pm_status)set_err(PM_EINVAL, "model projection / feature count mismatch");
    if (nv == 0) return PM_OK;
    DeviceGuard g(c->device);
    return (pm_status)run_host(c, v, nv, nullptr, m, t);
}

pm_status pm_count_device(pm_ctx *c, const pm_variant *d_v, size_t nv, pm_counts *d_counts,
                          const pm_model *m, double *d_t, int32_t *d_status, void *stream) {
    if (!c || (!d_v && nv) || (!d_status && nv)) return (pm_status)set_err(PM_EINVAL, "null argument");
    if (nv > PM_BATCH_MAX) return (pm_status)set_err(PM_EINVAL, "batch larger than PM_BATCH_MAX");
    if (m && (pm::nfeat(m->proj) < 0 || (int)m->nfeat != pm::nfeat(m->proj)))
        return (pm_status)set_err(PM_EINVAL, "model projection / feature count mismatch");
    if (nv == 0) return PM_OK;
    DeviceGuard g(c->device);
    int st = grow_cap(c, nv);
    if (st) return (pm_status)st;
    hipStream_t s = (hipStream_t)stream;  // NULL: HIP's null stream
    if ((st = arena_enter(c, s))) return (pm_status)st;
    st = pm::launch_batch(c->ar, c->sched, (int)nv, d_v, d_counts, (m && d_t) ? m : nullptr, d_t, d_status, s, c->n_cu,
                          c->next_events(), c->nmarks());
    if (st) return (pm_status)set_err(st, "counter launch failed");
    return (pm_status)arena_leave(c, s);
}

pm_status pm_count_device_noalloc(pm_ctx *c, const pm_variant *d_v, size_t nv,
                                  pm_counts *d_counts, const pm_model *m, double *d_t,
                                  int32_t *d_status, void *stream) {
    if (!c || (!d_v && nv) || (!d_status && nv)) return (pm_status)set_err(PM_EINVAL, "null argument");
    if (nv > PM_NOALLOC_MAX_VARIANTS)
        return (pm_status)set_err(PM_EINVAL, "batch of " + std::to_string(nv) +
                                                 " variants exceeds PM_NOALLOC_MAX_VARIANTS (" +
                                                 std::to_string(PM_NOALLOC_MAX_VARIANTS) + ")");
    if (m && (pm::nfeat(m->proj) < 0 || (int)m->nfeat != pm::nfeat(m->proj)))
        return (pm_status)set_err(PM_EINVAL, "model projection / feature count mismatch");
    if (nv == 0) return PM_OK;
    if (c->device < 0 || c->device >= noalloc::MAX_DEVICES || !noalloc::g_dev[c->device].ptr)
        return (pm_status)set_err(PM_EDEVICE, "scratch array not set up on this device");
    DeviceGuard g(c->device);
    noalloc::Dev &D = noalloc::g_dev[c->device];
    pm::Arena ar = noalloc::arena(D.ptr, D.parity);
    const int st = pm::launch_batch(ar, c->sched, (int)nv, d_v, d_counts, (m && d_t) ? m : nullptr,
                                    d_t, d_status, (hipStream_t)stream, c->n_cu, nullptr, 0);
    D.parity = ar.parity;  // the launch flipped it
    if (st) return (pm_status)set_err(st, "counter launch failed");
    return PM_OK;
}

pm_status pm_qpoly_derive(pm_ctx *c, const pm_variant *base, uint32_t fields, int64_t scale,
                          int32_t period, int64_t x0, pm_qpoly *out) {
    if (!c || !base || !out) return (pm_status)set_err(PM_EINVAL, "null argument");
    if (fields == 0 || fields > 7 || scale < 1 || period < 1 || period > PM_QPOLY_MAXPERIOD ||
        x0 < 1)
        return (pm_status)set_err(PM_EINVAL, "qpoly: fields 1..7, scale >= 1, period 1..64, x0 >= 1");
    constexpr int DEG = PM_QPOLY_DEGREE, NQ = PM_QPOLY_DEGREE + 3;
    const int64_t xmax = x0 + (int64_t)period * NQ;
    if (xmax > (int64_t)1 << 40 || scale > ((int64_t)1 << 40) / xmax)
        return (pm_status)set_err(PM_EINVAL, "qpoly: sizes too large");
    std::vector<pm_variant> vs((size_t)period * NQ);
    for (int r = 0; r < period; r++)
        for (int q = 0; q < NQ; q++) {
            pm_variant v = *base;
            const int64_t x = x0 + r + (int64_t)period * q;
            for (int i = 0; i < 3; i++)
                if ((fields >> i) & 1) v.n[i] = scale * x;
            vs[(size_t)r * NQ + q] = v;
        }
    std::vector<pm_counts> cnt(vs.size());
    const pm_status st = pm_count(c, vs.data(), vs.size(), cnt.data());
    if (st != PM_OK) return st;
    std::memset(out, 0, sizeof(*out));
    out->base = *base;
    out->fields = fields;
    out->period = period;
    out->scale = scale;
    out->x0 = x0;
    for (int r = 0; r < period; r++)
        for (int k = 0; k < PM_NCOUNT; k++) {
            // forward differences in q, exact in 128 bits
            __int128 d[NQ];
            for (int q = 0; q < NQ; q++) d[q] = cnt[(size_t)r * NQ + q].c[k];
            for (int ord = 0; ord <= DEG + 1; ord++) {
                if (ord <= DEG) {
                    if (d[0] > INT64_MAX || d[0] < INT64_MIN)
                        return (pm_status)set_err(PM_EOVERFLOW, "qpoly: coefficient beyond int64");
                    out->coef[r][ord][k] = (int64_t)d[0];
                } else if (d[0] != 0 || d[1] != 0) {
                    return (pm_status)set_err(
                        PM_EINVAL, "qpoly: count slot " + std::to_string(k) + " at residue " +
                                       std::to_string(r) + " is no polynomial of degree <= " +
                                       std::to_string(DEG) + " in q (period " +
                                       std::to_string(period) + " from x0 " + std::to_string(x0) + ")");
                }
                for (int q = 0; q + ord + 1 < NQ; q++) d[q] = d[q + 1] - d[q];
            }
        }
    return PM_OK;
}

pm_status pm_qpoly_eval(const pm_qpoly *qp, int64_t x, pm_counts *out) {
    if (!qp || !out) return (pm_status)set_err(PM_EINVAL, "null argument");
    if (qp->period < 1 || qp->period > PM_QPOLY_MAXPERIOD)
        return (pm_status)set_err(PM_EINVAL, "qpoly: not derived");
    if (x < qp->x0) return (pm_status)set_err(PM_EINVAL, "qpoly: x below x0");
    if (x - qp->x0 > ((int64_t)1 << 50)) return (pm_status)set_err(PM_EOVERFLOW, "qpoly: x too large");
    const int64_t r = (x - qp->x0) % qp->period, q = (x - qp->x0) / qp->period;
    // C(q, k) for k = 0 .. PM_QPOLY_DEGREE
    __int128 b[PM_QPOLY_DEGREE + 1];
    b[0] = 1;
    for (int k = 1; k <= PM_QPOLY_DEGREE; k++) b[k] = b[k - 1] * (q - (k - 1)) / k;
    for (int k = 0; k < PM_NCOUNT; k++) {
        __int128 v = 0, t;
        bool ovf = false;
        for (int j = 0; j <= PM_QPOLY_DEGREE; j++) {
            ovf |= __builtin_mul_overflow((__int128)qp->coef[r][j][k], b[j], &t);
            ovf |= __builtin_add_overflow(v, t, &v);
        }
        if (ovf || v > INT64_MAX || v < INT64_MIN)
            return (pm_status)set_err(PM_EOVERFLOW, "qpoly: count beyond int64 at this size");
        out->c[k] = (int64_t)v;
    }
    return PM_OK;
}

pm_status pm_qpoly_eval_many(const pm_qpoly *qp, const int64_t *xs, size_t nx, pm_counts *out) {
    if (!qp || (nx && (!xs || !out))) return (pm_status)set_err(PM_EINVAL, "null argument");
    for (size_t i = 0; i < nx; i++) {
        const pm_status st = pm_qpoly_eval(qp, xs[i], &out[i]);
        if (st != PM_OK) return st;
    }
    return PM_OK;
}

pm_status pm_reserve(pm_ctx *c, size_t nv, size_t bitmap_bytes) {
    if (!c) return (pm_status)set_err(PM_EINVAL, "null context");
    if (nv > PM_BATCH_MAX) return (pm_status)set_err(PM_EINVAL, "batch larger than PM_BATCH_MAX");
    DeviceGuard g(c->device);
    int st = grow_cap(c, nv);
    if (st) return (pm_status)st;
    return (pm_status)grow_bitmap(c, (bitmap_bytes + 7) / 8);
}

pm_status pm_profile(pm_ctx *c, int enable) {
    if (!c) return (pm_status)set_err(PM_EINVAL, "null context");
    if (enable < 0 || enable > 2) return (pm_status)set_err(PM_EINVAL, "profile mode is 0, 1 or 2");
    c->profile = enable;
    c->pcount = 0;
    c->pseen = 0;
    return PM_OK;
}

pm_status pm_profile_sample(pm_ctx *c, int every) {
    if (!c || every < 1) return (pm_status)set_err(PM_EINVAL, "sampling period is at least 1");
    c->pevery = every;
    c->pseen = 0;
    return PM_OK;
}

pm_status pm_set_schedule(pm_ctx *c, const pm_schedule *s) {
    if (!c || !s) return (pm_status)set_err(PM_EINVAL, "null argument");
    if (s->inblock_items < 0 || s->inblock_items > (1 << 20) || s->fused_items < 0 ||
        s->fused_items > (1 << 24) || s->tail_wgs_per_cu < 1 || s->tail_wgs_per_cu > 32 ||
        s->reserved != 0)
        return (pm_status)set_err(PM_EINVAL, "schedule value out of range");
    c->sched.inblock_items = s->inblock_items;
    c->sched.fused_items = s->fused_items;
    c->sched.tail_wgs_per_cu = s->tail_wgs_per_cu;
    return PM_OK;
}

pm_status pm_get_schedule(pm_ctx *c, pm_schedule *s) {
    if (!c || !s) return (pm_status)set_err(PM_EINVAL, "null argument");
    s->inblock_items = c->sched.inblock_items;
    s->fused_items = c->sched.fused_items;
    s->tail_wgs_per_cu = c->sched.tail_wgs_per_cu;
    s->reserved = 0;
    return PM_OK;
}

pm_status pm_profile_read(pm_ctx *c, double *ms, int *nbatch) {
    if (!c || !ms) return (pm_status)set_err(PM_EINVAL, "null argument");
    DeviceGuard g(c->device);
    int n = c->pcount;
    for (int i = 0; i < PM_NPHASE; i++) ms[i] = 0;
    const int nph = c->nmarks() - 1;  // phases recorded
    for (int b = 0; b < n; b++) {
        hipEvent_t *e = &c->pev[(size_t)b * (PM_NPHASE + 1)];
        if (hipEventSynchronize(e[nph]) != hipSuccess)
            return (pm_status)set_err(PM_EDEVICE, "event wait failed");
        for (int i = 0; i < nph; i++) {
            float t = 0;
            if (hipEventElapsedTime(&t, e[i], e[i + 1]) != hipSuccess)
                return (pm_status)set_err(PM_EDEVICE, "no timing recorded");
            ms[i] += t;
        }
    }
    if (n)
        for (int i = 0; i < PM_NPHASE; i++) ms[i] /= n;
    if (nbatch) *nbatch = n;
    c->pcount = 0;
    c->pseen = 0;
    return PM_OK;
}

pm_status pm_batch_stats(pm_ctx *c, int64_t *stats) {
    if (!c || !stats || !c->ar.meta) return (pm_status)set_err(PM_EINVAL, "no batch has run");
    DeviceGuard g(c->device);
    int64_t m[pm::META_WORDS];
    if (hipStreamSynchronize(c->stream) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(m, c->ar.meta + pm::META_WORDS * (c->ar.parity ^ 1), sizeof m,
                  hipMemcpyDeviceToHost) != hipSuccess)
        return (pm_status)set_err(PM_EDEVICE, "stats copy failed");
    for (int k = 0; k < 8; k++) stats[k] = 0;
    stats[0] = m[pm::M_CHUNKS] & pm::LIST_OFF_MASK;
    stats[1] = m[pm::M_USED];
    stats[2] = m[pm::M_SEGS] & pm::LIST_OFF_MASK;
    stats[3] = m[pm::M_DEFER];
    stats[4] = m[pm::M_WORDS];
    return PM_OK;
}

pm_status pm_bitmap_bytes(const pm_variant *v, size_t *bytes) {
    if (!bytes) return (pm_status)set_err(PM_EINVAL, "null out");
    int st = validate(v);
    if (st) return (pm_status)st;
    *bytes = (size_t)g_hb.prog->bitmap_words * 8;
    return PM_OK;
}

pm_status pm_features(const pm_counts *cnt, uint32_t proj, double *f, uint32_t *nf) {
    if (!cnt || !f) return (pm_status)set_err(PM_EINVAL, "null argument");
    int n = pm::features(cnt->c, proj, f);
    if (n < 0) return (pm_status)set_err(PM_EINVAL, "unknown projection");
    if (nf) *nf = (uint32_t)n;
    return PM_OK;
}

pm_status pm_fit(const pm_counts *P, const double *T, size_t nrows, uint32_t proj, pm_model *out,
                 double *cond, double *resid, uint32_t *rank) {
    int st = pm::fit_model(P, T, nrows, proj, out, cond, resid, rank);
    if (st == PM_EINVAL) return (pm_status)set_err(st, "fit: bad projection, empty input or non-positive time");
    if (st == PM_ERANK) return (pm_status)set_err(st, "fit: no non-zero feature column");
    return (pm_status)st;
}

pm_status pm_buffers(const pm_variant *v, size_t *bytes, uint32_t *role, uint32_t *nbufs) {
    if (!bytes || !role || !nbufs) return (pm_status)set_err(PM_EINVAL, "null argument");
    int st = validate(v);
    if (st) return (pm_status)st;
    return (pm_status)pm::buffers(*v, bytes, role, nbufs);
}

pm_status pm_launch(pm_ctx *c, const pm_variant *v, void *const *bufs, const size_t *bytes,
                    uint32_t nbufs, void *stream) {
    if (!c) return (pm_status)set_err(PM_EINVAL, "null context");
    int st = validate(v);
    if (st) return (pm_status)st;
    st = check_bufs(v, bufs, bytes, nbufs);
    if (st) return (pm_status)st;
    DeviceGuard g(c->device);
    st = pm::launch(*v, bufs, (hipStream_t)stream);  // NULL: HIP's null stream
    if (st) return (pm_status)set_err(st, "kernel launch failed");
    return PM_OK;
}

pm_status pm_measure(pm_ctx *c, const pm_variant *v, void *const *bufs, const size_t *bytes,
                     uint32_t nbufs, void *stream, int warmup, int reps, double *t_reps,
                     double *t_min) {
    return (pm_status)measure_impl(c, v, bufs, bytes, nbufs, stream, warmup, reps, -1.0, t_reps,
                                   t_min, nullptr, nullptr);
}

pm_status pm_measure_until(pm_ctx *c, const pm_variant *v, void *const *bufs, const size_t *bytes,
                           uint32_t nbufs, void *stream, int warmup, int reps, double deadline_s,
                           double *t_reps, double *t_min, int32_t *reps_done, uint32_t *flags) {
    return (pm_status)measure_impl(c, v, bufs, bytes, nbufs, stream, warmup, reps, deadline_s,
                                   t_reps, t_min, reps_done, flags);
}

pm_status pm_launch_floor(pm_ctx *c, void *stream, double *t_sec) {
    if (!c || !t_sec) return (pm_status)set_err(PM_EINVAL, "null argument");
    // the empty kernel: one work-group of 64 work-items
    pm_variant v{};
    v.family = PM_FAM_EMPTY;
    v.n[0] = 8;
    v.wg[0] = 8;
    v.wg[1] = 8;
    const double keep = c->launch_floor;
    double t = 0;
    int st = measure_impl(c, &v, nullptr, nullptr, 0, stream, 4, 26, -1.0, nullptr, &t, nullptr,
                          nullptr);
    if (st) {
        c->launch_floor = keep;
        return (pm_status)st;
    }
    c->launch_floor = t;
    *t_sec = t;
    return PM_OK;
}

// ------------------------------------------------------------- testing ---
pm_status pm_count_host(const pm_variant *v, pm_counts *out, int64_t *foot) {
    if (!v || !out) return (pm_status)set_err(PM_EINVAL, "null argument");
    int st = pm::count_host(*v, out, foot, false);
    if (st) set_err(st, status_name(st));
    return (pm_status)st;
}

pm_status pm_count_host_seq(const pm_variant *v, pm_counts *out, int64_t *foot) {
    if (!v || !out) return (pm_status)set_err(PM_EINVAL, "null argument");
    int st = pm::count_host(*v, out, foot, true);
    if (st) set_err(st, status_name(st));
    return (pm_status)st;
}

}  // extern "C"
