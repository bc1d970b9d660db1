/*
 * pm.h -- C ABI of libpm: a hardware-fitted linear run-time model for
 * MI355X (gfx950) after Stevens and Kloeckner, "A Unified, Hardware-Fitted,
 * Cross-GPU Performance Model" (arXiv 1604.04997).
 *
 * The model (Sec. 2):  T(n) ~ sum_i alpha_i p_i(n).  The p_i are operation
 * counts of a kernel variant -- global accesses by size, direction and
 * amortized stride class (Sec. 2.1), LDS accesses, flops by kind and dtype
 * (Sec. 2.2), barriers (Sec. 2.3), work-groups and a constant (Sec. 2.4).
 * The alpha_i are fitted once per device to measured run times of
 * performance-instructive kernels (Sec. 4).
 *
 * Conventions for every call:
 *   - return value: pm_status, 0 on success, < 0 on error; no C++ exception
 *     crosses this boundary; pm_last_error() gives a message for the last
 *     failing call on the calling thread (valid until its next call);
 *   - every array argument is owned by the caller; the library never frees
 *     or keeps caller memory past the call (the *_device calls read and
 *     write caller device memory asynchronously on the caller's stream,
 *     until that stream reaches the point where the call was enqueued);
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device allocations on the context's device;
 *   - a context is used by one thread at a time.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PM_OK = 0,
    PM_EINVAL = -1,     /* bad argument or variant descriptor */
    PM_ENOMEM = -2,     /* device memory (or the context's HBM budget) exhausted */
    PM_EDEVICE = -3,    /* a HIP runtime call failed */
    PM_ERANK = -4,      /* fit: no non-zero feature column */
    PM_EOVERFLOW = -5,  /* a count does not fit in int64 */
    PM_ETIMEDOUT = -6,  /* measure: deadline passed */
    PM_EBUSY = -7       /* context in use */
} pm_status;

/* Kernel families (each is a hand-written HIP kernel of the suite). */
enum {
    PM_FAM_STREAM = 0,    /* global-memory stream (Sec. 4.1 stride-1/-2/-3 classes) */
    PM_FAM_LDS = 1,       /* LDS reads / writes at a bank stride */
    PM_FAM_FMA = 2,       /* FMA chains (Sec. 4.1 arithmetic operations) */
    PM_FAM_RSQRT = 3,     /* rsqrt chains */
    PM_FAM_BARRIER = 4,   /* barrier loops (Sec. 2.3) */
    PM_FAM_EMPTY = 5,     /* empty kernel (Sec. 4.1, launch overhead) */
    PM_FAM_MATMUL = 6,    /* tiled / naive matrix multiplication */
    PM_FAM_TRANSPOSE = 7, /* LDS-tiled / naive transpose */
    PM_FAM_STENCIL = 8,   /* 5-point finite difference stencil (Sec. 5) */
    PM_FAM_NBODY = 9,     /* all-pairs n-body sum of 1/r (Sec. 5) */
    PM_FAM_ARITH = 10,    /* division / exponential chains (Sec. 4.1 arithmetic operations) */
    PM_FAM_CONV = 11,     /* three 7x7 filters over three RGB images (Sec. 5) */
    PM_NFAMILY = 12
};
enum { PM_F32 = 0, PM_F64 = 1 };
/* op values per family */
enum { PM_STREAM_LOAD = 0, PM_STREAM_STORE = 1, PM_STREAM_COPY = 2,
       PM_STREAM_ADD4 = 3, PM_STREAM_FILLED = 4, PM_STREAM_AXPBY = 5 };
enum { PM_ARITH_DIV = 0, PM_ARITH_EXP = 1 };
enum { PM_LDS_READ = 0, PM_LDS_WRITE = 1 };
enum { PM_MATMUL_TILED = 0, PM_MATMUL_NAIVE = 1 };
enum { PM_TRANSPOSE_TILED = 0, PM_TRANSPOSE_NAIVE_WC = 1, PM_TRANSPOSE_NAIVE_RC = 2 };

/*
 * One kernel variant: family + parameters (all sizes in elements).
 *   STREAM    n[0] work-items (multiple of wg[0]), wg[0], stride = lane
 *             stride s, gstride = group stride,
 *             vec = elements per access (1,2,4; 16 bytes max),
 *             reps = accesses per work-item U.  Element of access u of
 *             work-item (g,l): vec*(((g*gs)*wg + l)*s + u*G*gs*wg*s).
 *             FILLED (Sec. 4.1 stride-2/-3 "filled" access, generalised):
 *             of every s cells (2 <= s <= 64) the first c = chains are
 *             read (1 <= c <= min(s, 5); 0 means c = s), group j = i +
 *             u*n of work-item i reading cells s*j .. s*j + c - 1, summed
 *             left to right into a running sum stored at out[i]; vec = 1,
 *             gstride = 1.  Utilization about c/s reaches every stride class
 *             of Sec. 2.1 ('k/q' with q = min(s, 4)).
 *   LDS       n[0] groups, wg[0], stride = bank stride b, reps = R,
 *             words = W (power of two, multiple of wg, <= 16384)
 *   FMA       dtype, n[0] work-items, wg[0], reps = F, chains = K (F%K==0,
 *             K in {1,2,4,8,16})
 *   RSQRT     n[0], wg[0], reps = F, chains = K (K in {1,2,4,8}); fp32
 *   BARRIER   n[0] groups, wg[0], reps = B
 *   EMPTY     n[0] = side of a virtual n x n matrix, wg[0] x wg[1]
 *   MATMUL    op, n[0..2] = n, m, l (C[n,l] = A[n,m] B[m,l], row-major),
 *             tile T in {8,16,32} (work-group T x T); fp32
 *   TRANSPOSE op, n[0] = n (n x n, row-major), tile T in {8,16,32}; fp32
 *   STENCIL   dtype, n[0] = interior side n (input (n+2)^2 with halo),
 *             tile T in {8,16,32}
 *             AXPBY: out = 0.75 x + (-1.25) y elementwise (vector scale
 *             and add, Sec. 4.1).
 *   NBODY     n[0] bodies (positions 3 x n column-major), wg[0] block size
 *             (64..1024, multiple of 64); fp32
 *   ARITH     op DIV: chains y = (k+1) / (y*y + 1); op EXP: y = exp(-(y*y));
 *             dtype, n[0] work-items, wg[0], reps = F, chains = K (as FMA)
 *   CONV      n[0] = output side n; tile T in {8,16} (work-group T x T);
 *             r[i][j][x][y] = sum_{u,v<7, c<3} img[i][x+6-u][y+6-v][c] *
 *             filt[j][u][v][c] for 3 images (n+6)^2 x 3 and 3 filters
 *             7 x 7 x 3, channel fastest; fp32
 * flags: PM_FLAG_BITMAP counts every footprint with bitmaps, also where
 * the interval form applies; PM_FLAG_ENUMERATE counts every guarded
 * component of two or more variables by enumerating its points (Alg. 1),
 * also where a closed form applies, and runs every such count job in the
 * chip-wide count kernel, also where the work-group that expanded the
 * descriptor could count it itself (same counts; both for cross-checks).
 * PM_FLAG_STREAMING (STREAM only, ignored elsewhere): every access of the
 * measured kernel carries the non-temporal cache hint; the counts do not
 * change (the properties of Sec. 3 do not see cache hints).
 * Unused fields must be zero.  `seed` is carried for the caller's records.
 */
#define PM_FLAG_BITMAP 1u
#define PM_FLAG_ENUMERATE 2u
#define PM_FLAG_STREAMING 4u
typedef struct {
    uint32_t family, dtype, op, flags;
    int64_t n[3];
    int32_t wg[2];
    int32_t tile, stride, gstride, vec, reps, chains, words, pad;
    uint64_t seed;
} pm_variant;

/*
 * Count vector (int64), layout:
 *   [0, 90)    global accesses [dir][size][class]: dir 0 load / 1 store,
 *              size 4/8/16 bytes, class 0 '0', 1 '1', 2..3 '1/2','2/2',
 *              4..6 '1/3'..'3/3', 7..10 '1/4'..'4/4', 11..14 '1/>4'..'4/>4'
 *   [90, 96)   LDS accesses [dir][size]
 *   [96, 108)  flops [kind][dtype]: kind add/sub, mul, div, exp/pow,
 *              special (rsqrt, sqrt, ...), fma; dtype f32, f64
 *   108 barriers summed over work-items, 109 barriers summed over groups,
 *   110 work-groups, 111 work-items
 *   [112, 154) the LDS accesses of [90, 96) again, split by bank-stride bin
 *              (Sec. 6.2: binning the stride of local memory access):
 *              [dir][size][bin], bin 0 a broadcast (the address does not
 *              move with the lane index), bins 1..6 an address that moves
 *              by s 4-byte words per lane with s odd, 2 x odd, 4 x odd,
 *              8 x odd, 16 x odd, a multiple of 32
 * pm_count_name() gives the name of each slot.
 */
#define PM_NCOUNT 154
typedef struct { int64_t c[PM_NCOUNT]; } pm_counts;

/* Feature projections of a count vector:
 *   PM_PROJ_P3    [global load+store bytes, fp32 FMAs, work-groups]
 *   PM_PROJ_P12   [1, work-groups, barriers (sum over work-items),
 *                  fp32 add+mul (FMA = 2), fp64 add+mul, special+div+exp,
 *                  LDS bytes, global-load bytes of classes 0,1,2/2,3/3,4/4,
 *                  global-store bytes of those classes, global-load bytes
 *                  of the other classes, global-store bytes of those,
 *                  min(stride-1 load bytes, stride-1 store bytes)]
 *   PM_PROJ_FULL  the paper's property list: 90 global access counts,
 *                  6 LDS counts, 10 flop counts (FMA = one add and one mul),
 *                  barriers, work-groups, const 1, 45 min(load, store)
 *                  counts per (size, class) -- 154 features
 *   PM_PROJ_EXT   PM_PROJ_FULL and three features for what the paper names
 *                  as extensions (Sec. 6, future work): arithmetic
 *                  instructions per resident work-item and global bytes per
 *                  resident work-item (a grid smaller than the GPU holds at
 *                  once runs as long as one work-item's chain:  x / min(WI,
 *                  PM_RESIDENT_WI)), and min(arithmetic instructions, global
 *                  bytes) for arithmetic overlapped with data motion --
 *                  157 features.  Arithmetic instructions: the sum of the
 *                  ten flop counts (an FMA once).
 *   PM_PROJ_BANK  PM_PROJ_EXT with its 6 LDS counts replaced by the 42 LDS
 *                  counts by bank-stride bin (slots [112, 154); Sec. 6.2)
 *                  -- 193 features: global (90), LDS by bin (42), then
 *                  PM_PROJ_EXT's features from the flops on (61). */
enum { PM_PROJ_P3 = 0, PM_PROJ_P12 = 1, PM_PROJ_FULL = 2, PM_PROJ_EXT = 3, PM_PROJ_BANK = 4 };
#define PM_RESIDENT_WI 524288 /* 256 CUs x 2048 work-items */
#define PM_NFEAT_MAX 200
typedef struct {
    uint32_t nfeat, proj;
    double alpha[PM_NFEAT_MAX]; /* seconds per unit of each feature */
} pm_model;

typedef struct pm_ctx pm_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the context may hold (0 = 64 GiB).  Owns its streams,
 * events and device arenas. */
pm_status pm_create(pm_ctx **out, int device, size_t hbm_budget_bytes);
void pm_destroy(pm_ctx *ctx);
const char *pm_last_error(void);

/* Name of count slot i (0 <= i < PM_NCOUNT), e.g. "gld.4.1/2", "fma.f32". */
pm_status pm_count_name(int i, char *buf, size_t cap);

/*
 * Kernel properties of nv variants (host arrays v[nv], out[nv]), counted on
 * the GPU by enumerating each variant's iteration domain: per instruction
 * the number of points of its guarded domain (Sec. 3.2, Alg. 1 and
 * Eq. opcount), per array the footprint and its gap-filled counterpart
 * (Alg. 2) that fix the amortized stride fraction (Sec. 2.1).  All nv
 * variants are counted together in one batched pass; the result does not
 * depend on nv or on the batch's composition.  Synchronous.
 * Errors: PM_EINVAL for an invalid descriptor (the message names the
 * variant), PM_EOVERFLOW if a count exceeds int64, PM_ENOMEM if a single
 * variant's footprint bitmaps exceed the HBM budget.
 */
pm_status pm_count(pm_ctx *ctx, const pm_variant *v, size_t nv, pm_counts *out);

/* pm_count followed by T = sum_i alpha_i f_i(counts) (Sec. 2) for each
 * variant, in FP64.  t_sec: host array [nv]. */
pm_status pm_predict(pm_ctx *ctx, const pm_model *m, const pm_variant *v,
                     size_t nv, double *t_sec);

/*
 * Device-resident batched path of pm_count / pm_predict (Sec. 3.2, Alg. 1
 * and 2, Eq. opcount; the prediction of Sec. 2): d_v[nv] (device) ->
 * d_counts[nv] (device, may be NULL), d_t[nv] (device, FP64 predictions
 * with model m; ignored if m or d_t is NULL), d_status[nv] (device int32: 0
 * or a pm_status per variant).  Enqueued on `hip_stream` (a hipStream_t,
 * used as given: NULL is HIP's null stream); returns without waiting.
 * Variants whose footprint bitmaps do not fit in the context's bitmap arena
 * get status PM_ENOMEM and are not counted; pm_reserve() sizes the arena.
 * At most PM_BATCH_MAX variants.  Batches of one context share its device
 * arena: a batch enqueued on another stream than the context's previous
 * batch first waits (hipStreamWaitEvent) for that batch, so calls on
 * different streams, and pm_count / pm_predict between them, are ordered
 * in the order they were made.
 */
#define PM_BATCH_MAX 65536
pm_status pm_count_device(pm_ctx *ctx, const pm_variant *d_v, size_t nv,
                          pm_counts *d_counts, const pm_model *m, double *d_t,
                          int32_t *d_status, void *hip_stream);

/*
 * pm_count_device for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the counter's working
 * memory in a fixed device array of the library (about 40 MB on every
 * device it runs on, held until the process ends) instead of the
 * context's arena.  Allocates nothing: no hipMalloc, hipFree or
 * allocating library call.  Arguments as pm_count_device; at most
 * PM_NOALLOC_MAX_VARIANTS variants (else PM_EINVAL, nothing enqueued);
 * variants whose footprint bitmaps do not fit in PM_NOALLOC_BITMAP_BYTES
 * (together with those of the variants before them in the batch) get
 * status PM_ENOMEM.  Every call on one GPU uses that GPU's one array: calls
 * that may overlap on the device (different streams with no order between
 * them) race, and the caller must order them.  The array keeps the last
 * call's contents; what a batch needs cleared it clears itself.  Asynchronous
 * on `hip_stream`, like pm_count_device.
 */
#define PM_NOALLOC_MAX_VARIANTS 1024
#define PM_NOALLOC_BITMAP_BYTES (16u << 20)
pm_status pm_count_device_noalloc(pm_ctx *ctx, const pm_variant *d_v, size_t nv,
                                  pm_counts *d_counts, const pm_model *m, double *d_t,
                                  int32_t *d_status, void *hip_stream);

/*
 * Counts as quasi-polynomials of one size, re-evaluated in O(1) (Sec. 3.2:
 * the counts are piecewise quasi-polynomials in the size parameters; Sec. 2:
 * once found they are cheaply re-evaluated for changed sizes).  Take the
 * variant `base` with each size field n[i] in `fields` (bit i) set to
 * scale * x.  For x >= x0 every count is then, on each residue
 * r = (x - x0) mod period, a polynomial of degree at most PM_QPOLY_DEGREE
 * in q = (x - x0) div period, written in the binomial basis:
 * count = sum_k coef[r][k] * C(q, k).
 * pm_qpoly_derive finds the coefficients from the counter itself: one
 * batched pm_count of the variants at x = x0 + r + period*q for every
 * residue r and q = 0 .. PM_QPOLY_DEGREE + 2, exact integer forward
 * differences in q, and a check that the differences of order
 * PM_QPOLY_DEGREE + 1 vanish at both extra points of every residue and
 * count.  PM_EINVAL (the message says which) for a bad argument, an invalid
 * variant at some x, or counts that are no such quasi-polynomial with this
 * period from x0; the status of pm_count otherwise.  `out` is caller-owned.
 * pm_qpoly_eval writes the counts at x (host, no GPU): PM_EINVAL for
 * x < x0, PM_EOVERFLOW when a count leaves int64.
 */
#define PM_QPOLY_MAXPERIOD 64
#define PM_QPOLY_DEGREE 3
typedef struct {
    pm_variant base;
    uint32_t fields;
    int32_t period;
    int64_t scale, x0;
    int64_t coef[PM_QPOLY_MAXPERIOD][PM_QPOLY_DEGREE + 1][PM_NCOUNT];
} pm_qpoly;
pm_status pm_qpoly_derive(pm_ctx *ctx, const pm_variant *base, uint32_t fields, int64_t scale,
                          int32_t period, int64_t x0, pm_qpoly *out);
pm_status pm_qpoly_eval(const pm_qpoly *qp, int64_t x, pm_counts *out);
/* pm_qpoly_eval at nx sizes xs[nx] (host) into out[nx]; stops at the first
 * failing size and returns its status. */
pm_status pm_qpoly_eval_many(const pm_qpoly *qp, const int64_t *xs, size_t nx, pm_counts *out);

/* Size the context's device arenas for batches of up to nv variants whose
 * footprint bitmaps total up to bitmap_bytes.  Fails with PM_ENOMEM beyond
 * the HBM budget. */
pm_status pm_reserve(pm_ctx *ctx, size_t nv, size_t bitmap_bytes);

/* Schedule of the batched counter: how a batch's work is split between
 * the work-group that expands each variant and the chip-wide kernels.
 * inblock_items: a variant (batches over 32) whose count jobs hold at most
 *   this many outer points is counted by its own 64-wide work-group; larger
 *   ones are handed on (0..2^20, default 4096);
 * fused_items: the same limit for batches of up to 32 variants, whose
 *   work-groups are 256 wide (0..2^24, default 2^20);
 * tail_wgs_per_cu: work-groups per compute unit of the chip-wide kernels
 *   (1..32, default 4).
 * Counts and predictions do not depend on it (integer sums); only the time
 * does.  pm_set_schedule returns PM_EINVAL for a value outside its range
 * and leaves the schedule unchanged; pm_get_schedule writes the current
 * one.  Both host calls; batches already launched keep their schedule. */
typedef struct {
    int64_t inblock_items;
    int64_t fused_items;
    int32_t tail_wgs_per_cu;
    int32_t reserved;  /* zero */
} pm_schedule;
pm_status pm_set_schedule(pm_ctx *ctx, const pm_schedule *s);
pm_status pm_get_schedule(pm_ctx *ctx, pm_schedule *s);

/* Per-kernel timing of the batched counter.  pm_profile(ctx, 1) starts a
 * timing window (pm_profile(ctx, 2): the same with events around the
 * expansion kernel only, ms[0]): every batch until pm_profile_read (at most
 * PM_PROFILE_MAX batches) takes HIP events at the start and end of its
 * kernels, recorded by the kernels' own dispatches (no packets of their
 * own on the stream), which bound its three phases: ms[0] the expansion kernel
 * (per-variant expansion, count and finish), ms[1] the time between the two
 * kernels (empty on the device path; in the synchronous host calls the
 * host's read of the expansion's statuses), ms[2] the chip-wide kernel for
 * the variants handed on (bitmap clearing, count and footprint chunks,
 * fill, finish).  pm_profile_read waits for the recorded batches and
 * writes the mean duration of each phase in milliseconds to
 * ms[PM_NPHASE] (host) and the number of batches to *nbatch; the window
 * then restarts.  pm_profile(ctx, 0) stops recording.  In the synchronous
 * host calls the chip-wide kernel runs only when the expansion handed
 * variants on; phases that did not run read zero.
 * pm_batch_stats writes, for the last batch, stats[0] work chunks,
 * stats[1] bitmap words cleared, stats[2] fill segments, stats[3] variants
 * handed on to the chip-wide kernel, stats[4] bitmap words requested
 * (host int64[8]); synchronous. */
#define PM_NPHASE 3
#define PM_PROFILE_MAX 4096
pm_status pm_profile(pm_ctx *ctx, int enable);
/* Events on one batch in `every` (>= 1, default 1) of a timing window, so
 * that a long run of batches carries the events' cost on a few of them
 * only; the means pm_profile_read gives are over the batches recorded. */
pm_status pm_profile_sample(pm_ctx *ctx, int every);
pm_status pm_profile_read(pm_ctx *ctx, double *ms, int *nbatch);
pm_status pm_batch_stats(pm_ctx *ctx, int64_t *stats);

/* Bytes of footprint bitmap one variant needs (host computation). */
pm_status pm_bitmap_bytes(const pm_variant *v, size_t *bytes);

/* Derived features of one count vector (host): f[*nfeat], the properties
 * p_i of Sec. 2 formed from the counts as in Sec. 4.2 (last paragraph):
 * global access counts by size, direction and stride class (Sec. 2.1), LDS
 * accesses and flops by kind and precision (Sec. 2.2), barriers (Sec. 2.3),
 * work-groups and the constant (Sec. 2.4), and the min(load, store) pairs
 * of Sec. 2.1, projected as `proj` describes (PM_PROJ_*).  *nfeat
 * (nullable) receives the number written.  PM_EINVAL for an unknown
 * projection. */
pm_status pm_features(const pm_counts *c, uint32_t proj, double *f,
                      uint32_t *nfeat);

/*
 * Fit (Sec. 4.3): the weights minimising sum_j (1 - sum_i a_i f_ji / T_j)^2
 * over nrows measured variants (counts P[nrows], run times T[nrows] in
 * seconds), by column-pivoted Householder QR in FP64 on the host.  Feature
 * columns that are zero in every row are left out and get weight 0.
 * out: the model; cond (nullable): |R_00| / |R_rr| of the kept columns;
 * resid (nullable, [nrows]): 1 - pred_j / T_j; rank (nullable).
 * PM_ERANK if no column is non-zero.
 */
pm_status pm_fit(const pm_counts *P, const double *T, size_t nrows,
                 uint32_t proj, pm_model *out, double *cond, double *resid,
                 uint32_t *rank);

/* Device buffers a variant's kernel takes: bytes[i] and role[i] (0 input,
 * 1 output, 2 input+output, 3 sentinel output that must stay unchanged),
 * *nbufs <= PM_MAXBUF. */
#define PM_MAXBUF 8
pm_status pm_buffers(const pm_variant *v, size_t *bytes, uint32_t *role,
                     uint32_t *nbufs);

/* Launch the variant's kernel once on `hip_stream` (async; NULL is HIP's
 * null stream).  bufs: device pointers as listed by pm_buffers, each at
 * least that many bytes. */
pm_status pm_launch(pm_ctx *ctx, const pm_variant *v, void *const *bufs,
                    const size_t *bytes, uint32_t nbufs, void *hip_stream);

/*
 * Measure (Sec. 4.2): `warmup` untimed launches, then `reps` launches each
 * timed with HIP events on `hip_stream` (NULL is HIP's null stream);
 * t_reps[reps] (nullable) receives
 * each time in seconds and *t_min the minimum.  Synchronous.
 */
pm_status pm_measure(pm_ctx *ctx, const pm_variant *v, void *const *bufs,
                     const size_t *bytes, uint32_t nbufs, void *hip_stream,
                     int warmup, int reps, double *t_reps, double *t_min);

/*
 * Launch overhead (Sec. 4.2: the empty kernel is run first on each GPU to
 * find it): the minimum over 26 timed launches, after 4 untimed ones, of
 * the empty kernel with one work-group of 64 work-items, on `hip_stream`.
 * *t_sec receives it in seconds and the context keeps it as its launch
 * floor for pm_measure_until.  Synchronous.
 */
pm_status pm_launch_floor(pm_ctx *ctx, void *hip_stream, double *t_sec);

/*
 * pm_measure with a deadline and the launch floor check.  Timed launches
 * are enqueued at most 4 ahead of the last one that completed.
 * deadline_s >= 0: once that much host wall time has passed since the
 * call began, no further launch is enqueued and the call returns
 * PM_ETIMEDOUT; launches already enqueued still run to completion on the
 * stream (the caller keeps its buffers alive until the stream reaches
 * them; the next measurement on the context waits for them).  deadline_s
 * < 0: no deadline.  *reps_done (nullable) receives the number of timed
 * launches that completed, t_reps[0 .. *reps_done) their times and *t_min
 * their minimum (0 if none).  *flags (nullable) receives
 * PM_MEASURE_BELOW_FLOOR when the context has a launch floor
 * (pm_launch_floor) and *t_min is below twice it: the kernel's own work
 * then takes less time than launching it, the regime Sec. 4.2 keeps
 * measurement and test sizes out of.
 */
#define PM_MEASURE_BELOW_FLOOR 1u
pm_status pm_measure_until(pm_ctx *ctx, const pm_variant *v, void *const *bufs,
                           const size_t *bytes, uint32_t nbufs, void *hip_stream,
                           int warmup, int reps, double deadline_s, double *t_reps,
                           double *t_min, int32_t *reps_done, uint32_t *flags);

#ifdef __cplusplus
}
#endif
#endif /* PM_H */
