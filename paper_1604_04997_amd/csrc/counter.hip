// GPU counter: kernel properties of a batch of variants (Sec. 3.2).
//
// Both first kernels expand a variant's descriptor in LDS with one thread
// per statement (desc.h: build_head, analyze_stmt, build_tail).
// k_fused     batches of up to FUSED_MAX_NV variants, one work-group each:
//             also runs the count jobs (guarded points per statement, Alg.
//             1) with all its threads and writes the count vector (Eq.
//             opcount) and the FP64 prediction.  A variant whose footprints
//             need bitmaps (or whose jobs exceed the schedule's item limit) is
//             handed on: its descriptor is copied to HBM, status PM_DEFER.
// k_build     larger batches, one 64-wide work-group per variant: counts
//             small count jobs itself and finishes those variants, hands the
//             others on with their descriptor and jobs in HBM.
// A variant handed on claims, with atomics, its bitmap words (PM_ENOMEM
// when they pass the arena's end) and entries in the chunk, segment and
// finish lists (counter.h).  For handed-on variants only, one chip-wide
// launch:
//   k_tail      wavefronts take work items by ticket: clear the used bitmap
//               words; count chunks (sums of inner interval lengths) and
//               footprint chunks (cell runs OR-ed into the bitmaps); fill
//               segments (|F| and |Fill|, F with every strided cell widened
//               to its run of stride*vec cells); the count vector and
//               prediction of each variant -- each item after the ones it
//               needs (per-variant completion counters)
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdlib>
#include <vector>

#include "counter.h"
#include "desc.h"

namespace pm {

constexpr int FUSED_THREADS = 256;
constexpr int FUSED_MAX_NV = 32;       // batches up to this size use k_fused

// Sums and scans over one wavefront's 64 lanes, every lane active, in the
// vector ALU (no ds_bpermute).  Across rows of 16 lanes: gfx950's
// v_permlane32_swap / v_permlane16_swap of a value with itself give every
// lane the lower and the upper of the two halves (rows) it pairs, whose sum
// is its own value plus its xor-32 (xor-16) partner's.  Inside a row, DPP
// row_ror:k gives lane i the value of lane (i - k) mod 16: once lanes that
// differ only in bits above k hold equal values, that is lane i xor k's.
// So xsum adds the same pairs in the same order as a xor butterfly over
// 32, 16, ..., 1 (bit for bit, also in floating point).  scan_incl:
// row_shr steps inside each row, then each row adds the totals of the rows
// below it through row_bcast:15 and row_bcast:31.
constexpr int DPP_ROW_SHR = 0x110, DPP_ROW_ROR = 0x120, DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;
template <int CTRL, int ROWMASK = 0xF>
__device__ inline uint64_t dpp64(uint64_t u) {  // lanes with no source, or in masked rows: 0
    constexpr bool zero_oob = ROWMASK == 0xF;
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWMASK, 0xF, zero_oob);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWMASK, 0xF, zero_oob);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
template <int CTRL>
__device__ inline double dpp_f64(double x) {
    return __longlong_as_double((long long)dpp64<CTRL>((uint64_t)__double_as_longlong(x)));
}
template <int HALF>  // 32: lanes l and l ^ 32; 16: lanes l and l ^ 16
__device__ inline void swap_pair(uint64_t u, uint64_t *lo_half, uint64_t *hi_half) {
    const uint32_t a = (uint32_t)u, b = (uint32_t)(u >> 32);
    if constexpr (HALF == 32) {
        const auto pa = __builtin_amdgcn_permlane32_swap(a, a, false, false);
        const auto pb = __builtin_amdgcn_permlane32_swap(b, b, false, false);
        *lo_half = ((uint64_t)pb[0] << 32) | pa[0];
        *hi_half = ((uint64_t)pb[1] << 32) | pa[1];
    } else {
        const auto pa = __builtin_amdgcn_permlane16_swap(a, a, false, false);
        const auto pb = __builtin_amdgcn_permlane16_swap(b, b, false, false);
        *lo_half = ((uint64_t)pb[0] << 32) | pa[0];
        *hi_half = ((uint64_t)pb[1] << 32) | pa[1];
    }
}
template <int HALF>
__device__ inline double pair_sum(double x) {
    uint64_t p, q;
    swap_pair<HALF>((uint64_t)__double_as_longlong(x), &p, &q);
    return __longlong_as_double((long long)p) + __longlong_as_double((long long)q);
}
template <int HALF>
__device__ inline int64_t pair_sum(int64_t x) {
    uint64_t p, q;
    swap_pair<HALF>((uint64_t)x, &p, &q);
    return (int64_t)p + (int64_t)q;
}
__device__ inline double xsum(double x) {
    x = pair_sum<32>(x);
    x = pair_sum<16>(x);
    x += dpp_f64<DPP_ROW_ROR + 8>(x);
    x += dpp_f64<DPP_ROW_ROR + 4>(x);
    x += dpp_f64<DPP_ROW_ROR + 2>(x);
    x += dpp_f64<DPP_ROW_ROR + 1>(x);
    return x;
}
__device__ inline int64_t xsum(int64_t x) {
    x = pair_sum<32>(x);
    x = pair_sum<16>(x);
    x += (int64_t)dpp64<DPP_ROW_ROR + 8>((uint64_t)x);
    x += (int64_t)dpp64<DPP_ROW_ROR + 4>((uint64_t)x);
    x += (int64_t)dpp64<DPP_ROW_ROR + 2>((uint64_t)x);
    x += (int64_t)dpp64<DPP_ROW_ROR + 1>((uint64_t)x);
    return x;
}
__device__ inline int64_t scan_incl(int64_t c) {  // lane j: the sum over lanes 0..j
    c += (int64_t)dpp64<DPP_ROW_SHR + 1>((uint64_t)c);
    c += (int64_t)dpp64<DPP_ROW_SHR + 2>((uint64_t)c);
    c += (int64_t)dpp64<DPP_ROW_SHR + 4>((uint64_t)c);
    c += (int64_t)dpp64<DPP_ROW_SHR + 8>((uint64_t)c);
    c += (int64_t)dpp64<DPP_BCAST15, 0xA>((uint64_t)c);  // rows 1 and 3: lane 15 of the row below
    c += (int64_t)dpp64<DPP_BCAST31, 0xC>((uint64_t)c);  // rows 2 and 3: lane 31
    return c;
}

// Expansion of one variant by a work-group (at least MAXSTMT threads; all
// call this): the first wavefront lays out the statements (affine forms
// spread over its lanes), thread si analyses
// statement si in job slots 2si and 2si+1, thread 0 finishes
// (build_slots_finish).  p and the NTEMP job buffers jt are in LDS, handed
// to the first statements that make jobs (the others make theirs in
// place); with `keep` (= jt) each statement's last job stays in its buffer
// (p->jtmp) instead of going to its slot in `jobs`; sh holds 2 + MAXSTMT
// ints.
constexpr int NTEMP = 4;
__device__ __forceinline__ int build_block(const pm_variant &v, Prog *p, Job *jobs, Job *jt,
                                           int *sh, Job *keep) {
    const int t = threadIdx.x;
    if (t < 64) {  // the first wavefront lays out the statements, all lanes together
        const int st = build_head<LaneAff>(v, p, jobs);
        if (t == 0) {
            sh[0] = st;
            sh[1 + MAXSTMT] = 0;  // temp buffers handed out
        }
    }
    __syncthreads();
    if (sh[0] != PM_OK) return sh[0];
    auto temp = [&]() -> Job * {
        const int k = atomicAdd(&sh[1 + MAXSTMT], 1);
        return k < NTEMP ? &jt[k] : nullptr;
    };
    if (t < p->nstmt) {
        int made;
        sh[1 + t] = analyze_stmt(p, t, jobs, temp, 2 * t, 2 * t + 2, PM_SEQ, &made, keep);
    }
    __syncthreads();
    if (t < 64) {
        // the usual case, decided by the lanes together: every statement
        // analysed in its two slots and no strided array, where the tail
        // only records the job slots (build_tail with no footprint to place)
        const int ns = p->nstmt, r = t < ns ? sh[1 + t] : PM_OK;
        const bool plain = __ballot(r != PM_OK) == 0 && __ballot(t < p->narr && p->arr[t].w) == 0;
        if (plain) {
            if (t == 0) {
                p->njob = 2 * ns;
                p->bitmap_words = 0;
                sh[0] = p->status;
            }
        } else if (t == 0) {
            sh[1 + MAXSTMT] = 0;  // the fallback hands the buffers out again
            sh[0] = build_slots_finish_seq(v, p, jobs, temp, sh + 1, keep, false);
        }
    }
    __syncthreads();
    if (sh[0] == PM_OK && t < 64) {
        // the job-chunk and fill-segment prefixes (build_tail's), as scans
        // over the first wavefront's lanes
        const int j = t;
        int64_t c = 0, g = 0;
        if (j < p->njob && p->jkind[j] != JOB_NONE)
            c = keep && p->jtmp[j] >= 0 ? keep[p->jtmp[j]].chunks : jobs[j].chunks;
        if (j < p->narr && p->arr[j].w && p->arr[j].words) g = p->arr[j].segs;
        c = scan_incl(c);
        g = scan_incl(g);
        if (j < MAXJOB) p->jobcum[j] = c;
        if (j < MAXARR) p->arrcum[j] = g;
        if (j == 63) p->chunks = c, p->segs = g;
    }
    __syncthreads();
    return sh[0];
}

// Tally entry k (0 .. NENT - MAXACC - 1) of statement s, as contrib()
// gives it for entry MAXACC + k: LDS accesses by direction and size, flops
// by kind and dtype, barriers, LDS sites by bank-stride bin.  The tallies
// are one block of words in the statement, so every lane takes the same
// path: one load, the slot and multiplier by selects.
static_assert(offsetof(Stmt, lsite) == offsetof(Stmt, lds) + 6 * 4 &&
              offsetof(Stmt, flop) == offsetof(Stmt, lsite) + MAXLSITE * 4 &&
              offsetof(Stmt, bar) == offsetof(Stmt, flop) + 12 * 4,
              "tally words of a statement: lds, lsite, flop, bar");
constexpr int NTALLY = NENT - MAXACC;
__device__ inline void tally_entry(const Stmt &s, int k, int *slot, int32_t *mult) {
    const int wi = k < 6 ? k : k < 18 ? k + MAXLSITE : k == 18 ? 6 + MAXLSITE + 12 : k - 13;
    const uint32_t w = ((const uint32_t *)&s.lds[0][0])[wi];
    const int dir = (w >> 19) & 1, z = (w >> 20) & 3, bin = (w >> 16) & 7;
    *slot = k < 6 ? C_LDS + k : k < 18 ? C_FLOP + k - 6 : k == 18 ? C_BARWI
          : C_LDSB + (dir * 3 + z) * NLBIN + bin;
    *mult = k < 19 ? (int32_t)w : (int32_t)(w & 0xffff);
}

struct FinShared {
    int64_t c[PM_NCOUNT];
    int64_t sc[MAXSTMT];
    int bad, big;
};

// Sums over a count vector that the projections use, by the 64 lanes (lane
// l takes slots l and l + 64; a butterfly combines them).  Every term is an
// integer, so while the sums stay below 2^53 they are exact and equal to
// the serial sums of feature_one.
struct Agg {
    double gb, ops, sp, ldsb, full0, full1, part0, part1, s10, s11;
};
__device__ inline double wave_sum(double x) { return xsum(x); }
__device__ Agg wave_aggregates(const int64_t *c, int l) {
    Agg a{};
    for (int k = l; k < C_LDSB; k += 64) {  // the binned LDS slots repeat [C_LDS, C_FLOP)
        const double x = (double)c[k];
        if (k < C_LDS) {
            const int d = k / 45, z = (k % 45) / NCLS, cl = k % NCLS;
            const double b = (z == 0 ? 4.0 : z == 1 ? 8.0 : 16.0) * x;
            const bool fu = full_use_class(cl);
            a.gb += b;
            a.full0 += (d == 0 && fu) ? b : 0.0;
            a.full1 += (d == 1 && fu) ? b : 0.0;
            a.part0 += (d == 0 && !fu) ? b : 0.0;
            a.part1 += (d == 1 && !fu) ? b : 0.0;
            a.s10 += (d == 0 && cl == 1) ? b : 0.0;
            a.s11 += (d == 1 && cl == 1) ? b : 0.0;
        } else if (k < C_FLOP) {
            const int z = (k - C_LDS) % 3;
            a.ldsb += (z == 0 ? 4.0 : z == 1 ? 8.0 : 16.0) * x;
        } else if (k < C_BARWI) {
            a.ops += x;
            const int kind = (k - C_FLOP) / 2;
            if (kind == K_SPEC || kind == K_DIV || kind == K_EXP) a.sp += x;
        }
    }
    a.gb = wave_sum(a.gb);
    a.ops = wave_sum(a.ops);
    a.sp = wave_sum(a.sp);
    a.ldsb = wave_sum(a.ldsb);
    a.full0 = wave_sum(a.full0);
    a.full1 = wave_sum(a.full1);
    a.part0 = wave_sum(a.part0);
    a.part1 = wave_sum(a.part1);
    a.s10 = wave_sum(a.s10);
    a.s11 = wave_sum(a.s11);
    return a;
}

// The two sums the extension features read (global bytes, arithmetic
// operations), by the 64 lanes: lane l takes global slots l and l + 64 and
// flop slot l; exact like wave_aggregates.
__device__ Agg wave_aggregates_ext(const int64_t *c, int l) {
    Agg a{};
    const double g0 = (double)c[l], g1 = l + 64 < C_LDS ? (double)c[l + 64] : 0.0;
    const int z0 = (l % 45) / NCLS, z1 = ((l + 64) % 45) / NCLS;
    a.gb = wave_sum((z0 == 0 ? 4.0 : z0 == 1 ? 8.0 : 16.0) * g0 +
                    (z1 == 0 ? 4.0 : z1 == 1 ? 8.0 : 16.0) * g1);
    a.ops = wave_sum(l < C_BARWI - C_FLOP ? (double)c[C_FLOP + l] : 0.0);
    return a;
}

// Feature i of PM_PROJ_FULL, PM_PROJ_EXT or PM_PROJ_BANK, equal to
// feature_one's bit for bit, on one path for every lane: the slots a
// feature reads and how it combines them are chosen by selects, so lanes
// on different kinds of feature do not diverge.  e0..e2: the extension
// features 154..156 (the same in every lane).
__device__ inline double feature_sel(const int64_t *c, uint32_t proj, int i, double e0,
                                     double e1, double e2) {
    int j = i, binned = 0;
    if (proj == PM_PROJ_BANK) {  // binned LDS counts at 90..131, EXT's features shifted past them
        binned = i >= 90 && i < 132;
        j = i < 90 ? i : binned ? 1000 : i - 36;
    }
    const bool g = j < 90, lds = j >= 90 && j < 96, fl = j >= 96 && j < 106;
    const bool mn = j >= 109 && j < 154;
    const int k = (j - 96) >> 1, d = (j - 96) & 1;
    const int z = (j - 109) / NCLS, cl = (j - 109) % NCLS;
    int A = g ? C_GACC + j : lds ? C_LDS + j - 90 : fl ? C_FLOP + 2 * k + d
          : j == 106 ? C_BARWI : j == 107 ? C_WG : mn ? C_GACC + z * NCLS + cl : 0;
    A = binned ? C_LDSB + i - 90 : A;
    const int B = fl ? C_FLOP + 2 * K_FMA + d : mn ? C_GACC + (3 + z) * NCLS + cl : 0;
    const int64_t a = c[A], b = c[B];
    double v = (double)a;
    v = fl && (k == K_ADD || k == K_MUL) ? v + (double)b : v;  // an FMA is an add and a mul
    v = mn ? (double)(a < b ? a : b) : v;
    v = j == 108 ? 1.0 : v;
    v = j == 154 ? e0 : j == 155 ? e1 : j == 156 ? e2 : v;
    return v;
}

// feature_one(c, proj, j), with the sums over many slots taken from `a`.
__device__ double feature_dev(const int64_t *c, uint32_t proj, int j, const Agg &a) {
    if (proj == PM_PROJ_BANK) {
        int slot = 0;
        j = bank_to_ext(j, &slot);
        if (j < 0) return (double)c[slot];
        proj = PM_PROJ_EXT;
    }
    if (proj == PM_PROJ_P3) return j == 0 ? a.gb : feature_one(c, proj, j);
    if (proj == PM_PROJ_P12) {
        switch (j) {
        case 5: return a.sp;
        case 6: return a.ldsb;
        case 7: return a.full0;
        case 8: return a.full1;
        case 9: return a.part0;
        case 10: return a.part1;
        case 11: return a.s10 < a.s11 ? a.s10 : a.s11;
        default: return feature_one(c, proj, j);
        }
    }
    if (proj == PM_PROJ_EXT && j >= 154) {
        const double wi = (double)(c[C_WI] < PM_RESIDENT_WI ? c[C_WI] : PM_RESIDENT_WI);
        if (j == 154) return wi > 0 ? a.ops / wi : 0.0;
        if (j == 155) return wi > 0 ? a.gb / wi : 0.0;
        return a.ops < a.gb ? a.ops : a.gb;
    }
    return feature_one(c, proj, j);
}

// Count vector and prediction of one variant by one work-group: every
// thread calls this, the first wavefront does the work.  Lanes take the
// statement counts, then the statements' contributions -- first their
// global accesses, then their other tallies, e = l, l + 64, ... in each --
// adding each non-zero one into its slot with an LDS atomic (exact: while
// every product is below 2^54 no sum of at most MAXSTMT*NENT of them can
// pass int64; larger products take exact per-slot sums with overflow
// checks).  Lane l then owns the features i = l (mod 64); the
// prediction's 64 partial sums meet in a butterfly, the order predict()
// fixes.  st != PM_OK: zero counts, prediction 0.
__device__ __forceinline__ int finalize_block(const Prog &p, const int64_t *jobres, const int64_t *F,
                              const int64_t *Fill, int st, FinShared &sh, pm_counts *out,
                              const pm_model &model, int has_model, double *pred) {
    const int t = threadIdx.x, l = t & 63;
    const bool w0 = t < 64;
    const int nst = st == PM_OK ? p.nstmt : 0;
    if (t == 0) sh.bad = sh.big = 0;
    if (w0)
        for (int k = l; k < PM_NCOUNT; k += 64) sh.c[k] = 0;
    if (w0 && l < nst && !stmt_count(p, l, jobres, &sh.sc[l])) sh.bad = 1;
    __syncthreads();
    if (w0 && st == PM_OK) {
        auto add = [&](int si, int slot, int32_t mult) {
            int64_t v;
            if (mul_ovf(sh.sc[si], (int64_t)mult, &v)) sh.bad = 1;
            else if (v >= (1ll << 54)) sh.big = 1;
            else if (v) atomicAdd((unsigned long long *)&sh.c[slot], (unsigned long long)v);
        };
        for (int e = l; e < nst * MAXACC; e += 64) {  // global accesses
            Contrib cc;
            if (contrib(p, e / MAXACC, e % MAXACC, F, Fill, &cc)) add(cc.stmt, cc.slot, cc.mult);
        }
        for (int e = l; e < nst * NTALLY; e += 64) {  // the other tallies
            const int si = e / NTALLY;
            int slot;
            int32_t mult;
            tally_entry(p.st[si], e % NTALLY, &slot, &mult);
            if (mult) add(si, slot, mult);
        }
        if (l == 0) {
            sh.c[C_WG] = p.n_wg;
            if (mul_ovf(p.n_wg, (int64_t)p.wg_size, &sh.c[C_WI])) sh.bad = 1;
        }
    }
    __syncthreads();
    if (w0 && st == PM_OK && sh.big)  // products this large: exact sums slot by slot
        for (int k = l; k < PM_NCOUNT; k += 64)
            if (k != C_BARWG && k != C_WG && k != C_WI && !slot_sum(p, k, F, Fill, sh.sc, &sh.c[k]))
                sh.bad = 1;
    __syncthreads();
    if (t == 0 && st == PM_OK) sh.c[C_BARWG] = p.wg_size ? tdiv(sh.c[C_BARWI], p.wg_size) : 0;
    __syncthreads();
    const int st2 = st == PM_OK && sh.bad ? PM_EOVERFLOW : st;
    if (out)
        for (int k = t; k < PM_NCOUNT; k += blockDim.x) out->c[k] = st2 == PM_OK ? sh.c[k] : 0;
    if (w0 && has_model && pred) {
        const uint32_t proj = model.proj;
        const bool sel = proj == PM_PROJ_FULL || proj == PM_PROJ_EXT || proj == PM_PROJ_BANK;
        const Agg a = sel ? wave_aggregates_ext(sh.c, l) : wave_aggregates(sh.c, l);
        const int nf = nfeat(proj) < (int)model.nfeat ? nfeat(proj) : (int)model.nfeat;
        double part = 0.0;
        if (st2 == PM_OK && sel) {
            const double wi = (double)(sh.c[C_WI] < PM_RESIDENT_WI ? sh.c[C_WI] : PM_RESIDENT_WI);
            const double e0 = wi > 0 ? a.ops / wi : 0.0, e1 = wi > 0 ? a.gb / wi : 0.0;
            const double e2 = a.ops < a.gb ? a.ops : a.gb;
            for (int i = l; i < nf; i += 64) part += model.alpha[i] * feature_sel(sh.c, proj, i, e0, e1, e2);
        } else if (st2 == PM_OK) {
            for (int i = l; i < nf; i += 64) part += model.alpha[i] * feature_dev(sh.c, proj, i, a);
        }
        part = xsum(part);
        if (t == 0) *pred = st2 == PM_OK ? part : 0.0;
    }
    return st2;
}

// Device buffers a kernel that hands variants on writes to.
struct HandOn {
    int64_t *meta;       // this batch's half
    int64_t *meta_next;  // the other half, cleared for the next batch by work-group 0
    int64_t *varoff;
    int64_t *vdone;      // per variant: chunks done, segments done
    int32_t *clist, *slist, *dlist;
    int64_t *cend, *send;
    int64_t arena_words;
    int64_t cap;  // list capacity (variants the arena holds)
};

// Hand variant i, whose program and jobs are in HBM, on to the chip-wide
// pipeline (one thread): claim its bitmap words and its work-list entries.
// Returns PM_DEFER, PM_ENOMEM when its bitmaps pass the arena's end, or
// PM_EOVERFLOW when it needs MAX_VARIANT_CHUNKS chunks or more.  (A list
// entry past the capacity, which only a meta half left dirty by an
// unfinished batch could give, is refused with PM_EDEVICE.)
__device__ __forceinline__ int hand_on(const Prog &P, int i, const HandOn &h) {
    if (P.chunks >= MAX_VARIANT_CHUNKS) return PM_EOVERFLOW;
    h.vdone[2 * (int64_t)i] = h.vdone[2 * (int64_t)i + 1] = 0;
    if (P.bitmap_words > 0) {
        const int64_t off = (int64_t)atomicAdd((unsigned long long *)&h.meta[M_WORDS],
                                               (unsigned long long)P.bitmap_words);
        if (off + P.bitmap_words > h.arena_words) return PM_ENOMEM;
        h.varoff[i] = off;
        atomicMax((unsigned long long *)&h.meta[M_USED], (unsigned long long)(off + P.bitmap_words));
    }
    if (P.chunks > 0) {
        const unsigned long long old = atomicAdd((unsigned long long *)&h.meta[M_CHUNKS],
                                                 (1ull << LIST_POS) + (unsigned long long)P.chunks);
        const int64_t pos = (int64_t)(old >> LIST_POS);
        if (pos >= h.cap) return PM_EDEVICE;
        h.clist[pos] = i;
        h.cend[pos] = (int64_t)(old & LIST_OFF_MASK) + P.chunks;
    }
    if (P.segs > 0) {
        const unsigned long long old = atomicAdd((unsigned long long *)&h.meta[M_SEGS],
                                                 (1ull << LIST_POS) + (unsigned long long)P.segs);
        const int64_t pos = (int64_t)(old >> LIST_POS);
        if (pos >= h.cap) return PM_EDEVICE;
        h.slist[pos] = i;
        h.send[pos] = (int64_t)(old & LIST_OFF_MASK) + P.segs;
    }
    const int64_t d = (int64_t)atomicAdd((unsigned long long *)&h.meta[M_DEFER], 1ull);
    if (d >= h.cap) return PM_EDEVICE;
    h.dlist[d] = i;
    return PM_DEFER;
}

// One variant per 64-wide work-group, expanded in LDS.  A variant without
// bitmaps whose count jobs hold at most `max_items` items (the schedule's
// in-block limit; and fit the LDS staging slots) is finished here: its jobs
// are counted by the work-group, then the count vector and prediction are
// written.  Any other is handed on with its program and jobs in HBM (status
// PM_DEFER, or PM_ENOMEM / PM_EOVERFLOW when it cannot be: zero outputs
// then).  The work-group's 10 KB of LDS allows 16 per CU; asking for four
// waves per SIMD keeps the registers within that occupancy too.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
k_build(int nv, const pm_variant *__restrict__ var, Prog *prog, Job *jobs, int32_t *status,
        int64_t *jobres, int64_t *foot, HandOn h, pm_counts *counts, pm_model model,
        int has_model, double *pred, int64_t max_items) {
    __shared__ Prog P;
    __shared__ union {
        Job jt[NTEMP];  // during the expansion; then the count jobs
        FinShared fin;  // for the count vector
    } U;
    __shared__ int64_t jr[MAXJOB];
    __shared__ int64_t zero[MAXARR];
    __shared__ int sh[2 + MAXSTMT];
    __shared__ int jid[NTEMP];   // count-job slots
    __shared__ int jbuf[NTEMP];  // the buffers they are counted from
    __shared__ int jfetch;       // of those, the first jfetch come from their slots
    const int i = blockIdx.x, t = threadIdx.x;
    if (i == 0 && t < META_WORDS) h.meta_next[t] = 0;
    if (i >= nv) return;
    if (t < MAXJOB) jr[t] = 0;
    if (t < MAXARR) zero[t] = 0;
    const pm_variant v = var[i];
    Job *vj = &jobs[(int64_t)i * MAXJOB];
    int st = build_block(v, &P, vj, U.jt, sh, U.jt);
    // Can this work-group finish the variant?  The lanes of the job slots
    // decide together (the work-group is one wavefront): at most NTEMP
    // count jobs holding at most max_items items.  Jobs still in a buffer
    // are counted there; the others are fetched from their slots into the
    // buffers no count job holds, the r-th fetched job (by slot) into the
    // r-th free buffer, and listed first.
    int ncj = -1;
    if (st == PM_OK && P.bitmap_words == 0 && !(P.flags & PM_FLAG_ENUMERATE)) {
        const bool cj = t < P.njob && P.jkind[t] == JOB_COUNT;
        const uint64_t m = __ballot(cj);
        const int tb = cj ? P.jtmp[t] : -1;
        int64_t items = 0;
        if (m) {  // (no count job: nothing to sum, nothing to place)
            items = cj ? (tb >= 0 ? U.jt[tb].items : vj[t].items) : 0;
            items = xsum(items);
        }
        const uint64_t fm = __ballot(cj && tb < 0);
        const int n = __popcll(m);
        if (!m && items <= max_items) {
            ncj = 0;
        } else if (n <= NTEMP && items <= max_items) {
            uint32_t held = 0;
#pragma unroll
            for (int b = 0; b < NTEMP; b++)
                if (__ballot(cj && tb == b)) held |= 1u << b;
            const uint64_t below = (1ull << t) - 1;
            const int nf = __popcll(fm);
            if (cj) {
                int pos = nf + __popcll(m & ~fm & below), buf = tb;
                if (tb < 0) {
                    pos = __popcll(fm & below);
                    for (int b = 0, r = pos; b < NTEMP; b++)
                        if (!((held >> b) & 1) && r-- == 0) buf = b;
                }
                jid[pos] = t;
                jbuf[pos] = buf;
            }
            if (t == 0) jfetch = nf;
            ncj = n;
        }
    }
    __syncthreads();
    if (ncj > 0) {
        constexpr int JW = sizeof(Job) / 8;
        for (int w = t; w < jfetch * JW; w += 64)  // count jobs not in a buffer
            ((uint64_t *)&U.jt[jbuf[w / JW]])[w % JW] =
                ((const uint64_t *)&vj[jid[w / JW]])[w % JW];
        __syncthreads();
        // the jobs' items as one range, spread over the lanes
        int64_t pre[NTEMP + 1];
        pre[0] = 0;
#pragma unroll
        for (int k = 0; k < NTEMP; k++) pre[k + 1] = pre[k] + (k < ncj ? U.jt[jbuf[k]].items : 0);
        int64_t s0[NTEMP] = {};
        for (int64_t x = t; x < pre[ncj]; x += 64) {
            int k = 0;
#pragma unroll
            for (int q = 1; q < NTEMP; q++) k += x >= pre[q];
            const int64_t c = count_item(U.jt[jbuf[k]], x - pre[k]);
#pragma unroll
            for (int q = 0; q < NTEMP; q++) s0[q] += q == k ? c : 0;
        }
#pragma unroll
        for (int q = 0; q < NTEMP; q++) {
            s0[q] = xsum(s0[q]);
            if (t == 0 && q < ncj) jr[jid[q]] = s0[q];
        }
        __syncthreads();
    }
    int sfin = st;  // finished here, or failed: zero outputs
    if (ncj < 0 && st == PM_OK) {  // handed on
        {  // jobs still in their buffers to their slots
            constexpr int JW = sizeof(Job) / 8;
            for (int w = t; w < NTEMP * JW; w += 64) {
                const int b = w / JW;
                int j = -1;
                for (int q = 0; q < P.njob; q++)
                    if (P.jtmp[q] == b) j = q;
                if (j >= 0) ((uint64_t *)&vj[j])[w % JW] = ((const uint64_t *)&U.jt[b])[w % JW];
            }
        }
        if (t < MAXJOB) jobres[(int64_t)i * MAXJOB + t] = 0;
        if (t < 2 * MAXARR) foot[(int64_t)i * MAXARR * 2 + t] = 0;
        // the program to HBM: header and used statements
        const int ns = P.nstmt < MAXSTMT ? P.nstmt : MAXSTMT;
        const size_t words = (offsetof(Prog, st) + (size_t)ns * sizeof(Stmt)) / 8;
        const uint64_t *src = (const uint64_t *)&P;
        uint64_t *dst = (uint64_t *)&prog[i];
        for (size_t w = t; w < words; w += 64) dst[w] = src[w];
        if (t == 0) sh[0] = hand_on(P, i, h);
        __syncthreads();
        sfin = sh[0];
        if (sfin == PM_DEFER) {
            if (t == 0) status[i] = sfin;
            return;
        }
    }
    const int s2 = finalize_block(P, jr, zero, zero, sfin, U.fin, counts ? &counts[i] : nullptr,
                                  model, has_model, pred ? &pred[i] : nullptr);
    if (t == 0) status[i] = s2;
}

// Sum of x over the work-group (FUSED_THREADS threads); all threads get it.
__device__ int64_t block_sum(int64_t x, int64_t *red) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = x;
    __syncthreads();
    int64_t t = 0;
    for (int k = 0; k < FUSED_THREADS / 64; k++) t += red[k];
    return t;
}

__global__ void __launch_bounds__(FUSED_THREADS)
k_fused(int nv, const pm_variant *__restrict__ var, Prog *prog, Job *jobs,
        int32_t *status, int64_t *jobres, int64_t *foot, HandOn h, pm_counts *counts,
        pm_model model, int has_model, double *pred, int64_t max_items) {
    __shared__ Prog P;
    __shared__ Job J[MAXJOB];
    __shared__ Job JT[NTEMP];
    __shared__ int64_t jr[MAXJOB];
    __shared__ int64_t fF[MAXARR], fFill[MAXARR];
    __shared__ int64_t red[FUSED_THREADS / 64];
    __shared__ FinShared fin;
    __shared__ int bsh[2 + MAXSTMT];
    __shared__ int st_sh;
    const int i = blockIdx.x;
    const int t = threadIdx.x;
    if (i == 0 && t < META_WORDS) h.meta_next[t] = 0;
    if (i >= nv) return;
    const pm_variant v = var[i];
    const int sb = build_block(v, &P, J, JT, bsh, nullptr);
    if (t == 0) {
        int st = sb;
        int64_t items = 0;
        for (int j = 0; j < P.njob; j++)
            if (P.jkind[j] != JOB_NONE) items += J[j].items;
        const bool enumerate = (P.flags & PM_FLAG_ENUMERATE) && items > 0;
        if (st == PM_OK && (P.bitmap_words > 0 || items > max_items || enumerate))
            st = PM_DEFER;
        st_sh = st;
    }
    if (t < MAXJOB) jr[t] = 0;
    if (t < MAXARR) fF[t] = fFill[t] = 0;
    __syncthreads();
    int st = st_sh;
    if (st == PM_DEFER) {  // hand the descriptor and zeroed sums on
        const uint64_t *src = (const uint64_t *)&P;
        uint64_t *dst = (uint64_t *)&prog[i];
        for (size_t k = t; k < sizeof(Prog) / 8; k += FUSED_THREADS) dst[k] = src[k];
        const uint64_t *js = (const uint64_t *)J;
        uint64_t *jd = (uint64_t *)&jobs[(size_t)i * MAXJOB];
        size_t nw = (size_t)P.njob * sizeof(Job) / 8;
        for (size_t k = t; k < nw; k += FUSED_THREADS) jd[k] = js[k];
        if (t < MAXJOB) jobres[(int64_t)i * MAXJOB + t] = 0;
        if (t < 2 * MAXARR) foot[(int64_t)i * MAXARR * 2 + t] = 0;
        if (t == 0) st_sh = hand_on(P, i, h);
        __syncthreads();
        st = st_sh;
        if (st == PM_DEFER) {
            if (t == 0) status[i] = st;
            return;
        }
    }
    if (st == PM_OK) {
        for (int j = 0; j < P.njob; j++) {
            if (P.jkind[j] != JOB_COUNT) continue;  // uniform over the group
            const Job &Jb = J[j];
            int64_t s0 = 0;
            for (int64_t it = t; it < Jb.items; it += FUSED_THREADS) s0 += count_item(Jb, it);
            s0 = block_sum(s0, red);
            if (t == 0) jr[j] = s0;
        }
        __syncthreads();
    }
    const int s2 = finalize_block(P, jr, fF, fFill, st, fin, counts ? &counts[i] : nullptr,
                                  model, has_model, pred ? &pred[i] : nullptr);
    if (t == 0) status[i] = s2;
}

// first index j in [0, n) with pref[j] > x (pref non-decreasing)
__device__ int64_t upper(const int64_t *pref, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (pref[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

struct DevOr {
    __device__ void operator()(uint64_t *p, uint64_t m) const {
        atomicOr((unsigned long long *)p, (unsigned long long)m);
    }
};

// Agent-scope counters through which the chip-wide kernel's work items
// hand their results on: a producer's writes are visible to a consumer
// that has seen its increment.
__device__ __forceinline__ void signal(int64_t *p) {
    __hip_atomic_fetch_add(p, (int64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_for(const int64_t *p, int64_t need) {
    while (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need)
        __builtin_amdgcn_s_sleep(2);
}

// Words of bitmap one clearing item zeroes, and one fill segment reads
// (64 lanes x FILL_WORDS_PER_LANE).
constexpr int64_t ZERO_WORDS = 4096;
constexpr int FILL_WORDS_PER_LANE = 64;
static_assert(64 * FILL_WORDS_PER_LANE == SEG_WORDS, "fill segment = one wavefront's words");

// Fill segment `local` of array `al` of variant v by one wavefront: |F|
// and |Fill| of its words (Fill: F with every strided cell widened to its
// run of w cells, including runs that start in earlier words) added to
// foot.
__device__ void fill_segment(const Prog &P, int al, int64_t local, const uint64_t *vb,
                             int64_t *foot_v, int l) {
    const ArrInfo &A = P.arr[al];
    const uint64_t *F = vb + A.f_off;
    const uint64_t *Bm = vb + A.b_off;
    const int64_t w = A.w;
    const int64_t k0 = local * SEG_WORDS;
    const int64_t k1 = k0 + SEG_WORDS < A.words ? k0 + SEG_WORDS : A.words;
    const int64_t a = k0 + (int64_t)l * FILL_WORDS_PER_LANE;
    const int64_t e = a + FILL_WORDS_PER_LANE < k1 ? a + FILL_WORDS_PER_LANE : k1;
    int64_t mylast = -1;
    for (int64_t k = e - 1; k >= a; k--) {
        const uint64_t b = Bm[k];
        if (b) {
            mylast = last_bit(b, k);
            break;
        }
    }
    // the last strided cell before the segment, within reach w
    const int64_t L = (w + 63) / 64 + 1;
    int64_t blast = -1;
    for (int64_t k = (k0 - L > 0 ? k0 - L : 0) + l; k < k0; k += 64) {
        const int64_t x = last_bit(Bm[k], k);
        if (x > blast) blast = x;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t y = __shfl_xor(blast, off);
        if (y > blast) blast = y;
    }
    // exclusive max-scan of mylast over the lanes
    int64_t incl = mylast;
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(incl, off);
        if (l >= off && y > incl) incl = y;
    }
    int64_t carry = __shfl_up(incl, 1);
    if (l == 0) carry = -1;
    if (blast > carry) carry = blast;
    unsigned long long pf = 0, pfill = 0;
    for (int64_t k = a; k < e; k++) {
        const uint64_t b = Bm[k];
        const uint64_t d = dilate_word(b, w) | carry_mask(carry, w, k);
        const uint64_t f = F[k];
        pf += __popcll(f);
        pfill += __popcll(f | d);
        if (b) carry = last_bit(b, k);
    }
    for (int off = 32; off > 0; off >>= 1) {
        pf += __shfl_xor(pf, off);
        pfill += __shfl_xor(pfill, off);
    }
    if (l == 0) {
        atomicAdd((unsigned long long *)&foot_v[al * 2], pf);
        atomicAdd((unsigned long long *)&foot_v[al * 2 + 1], pfill);
    }
}

// The chip-wide pass over the variants the expansion kernel handed on, in
// one launch of one-wavefront work-groups.  Every wavefront takes work
// items by ticket (meta[M_TICKET]) until the tickets run out:
//   [0, Z)             clear ZERO_WORDS of the bitmap words the batch uses
//   [Z, Z+C)           count and footprint chunks (footprint chunks first
//                      wait until the clearing is done)
//   [Z+C, Z+C+S)       fill segments (each waits until its variant's
//                      chunks are done)
//   [Z+C+S, Z+C+S+D)   finish a variant: count vector and prediction
//                      (waits until its chunks and segments are done)
// A wavefront only ever waits for items with smaller tickets, which
// wavefronts that are already running hold and finish without waiting
// for larger ones, so every wait ends and every wavefront exits.
__global__ void __launch_bounds__(64)
k_tail(const Prog *prog, const Job *jobs, const int32_t *clist, const int64_t *cend,
       const int32_t *slist, const int64_t *send, const int32_t *dlist, const int64_t *varoff,
       uint64_t *bitmap, int64_t *jobres, int64_t *foot, int64_t *vdone, int32_t *status,
       pm_counts *counts, pm_model model, int has_model, double *pred, int64_t *meta,
       int64_t cap, int64_t arena_words) {
    __shared__ FinShared fin;
    __shared__ int64_t Fs[MAXARR], Fills[MAXARR];
    const int l = threadIdx.x;
    // this batch's totals (written by the expansion kernel, an earlier launch)
    int64_t used = meta[M_USED] < arena_words ? meta[M_USED] : arena_words;
    const int64_t Z = (used + ZERO_WORDS - 1) / ZERO_WORDS;
    int64_t nc = (int64_t)((unsigned long long)meta[M_CHUNKS] >> LIST_POS);
    if (nc > cap) nc = cap;
    const int64_t C = nc ? cend[nc - 1] : 0;
    int64_t ns = (int64_t)((unsigned long long)meta[M_SEGS] >> LIST_POS);
    if (ns > cap) ns = cap;
    const int64_t S = ns ? send[ns - 1] : 0;
    const int64_t D = meta[M_DEFER] < cap ? meta[M_DEFER] : cap;
    const int64_t total = Z + C + S + D;
    if (total == 0) return;
    for (;;) {
        int64_t tk = 0;
        if (l == 0)
            tk = (int64_t)atomicAdd((unsigned long long *)&meta[M_TICKET], 1ull);
        tk = __shfl(tk, 0);
        if (tk >= total) return;
        if (tk < Z) {  // clear
            const int64_t w0 = tk * ZERO_WORDS;
            const int64_t w1 = w0 + ZERO_WORDS < used ? w0 + ZERO_WORDS : used;
            for (int64_t k = w0 + l; k < w1; k += 64) bitmap[k] = 0;
            __syncthreads();
            if (l == 0) signal(&meta[M_ZDONE]);
            continue;
        }
        tk -= Z;
        if (tk < C) {  // chunk -> list entry -> variant -> job
            const int64_t e = upper(cend, nc, tk);
            const int64_t v = clist[e];
            int64_t local = tk - (e ? cend[e - 1] : 0);
            const int64_t *cum = prog[v].jobcum;
            int jl = 0;
            while (cum[jl] <= local) jl++;
            local -= jl ? cum[jl - 1] : 0;
            const int64_t j = v * MAXJOB + jl;
            const Job &J = jobs[j];
            const int64_t it0 = local * J.chunk_items;
            const int64_t it1 = it0 + J.chunk_items < J.items ? it0 + J.chunk_items : J.items;
            if (J.kind == JOB_COUNT) {
                int64_t s = 0;
                for (int64_t it = it0 + l; it < it1; it += 64) s += count_item(J, it);
                for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
                if (l == 0 && s) atomicAdd((unsigned long long *)&jobres[j], (unsigned long long)s);
            } else {
                if (l == 0) wait_for(&meta[M_ZDONE], Z);
                __syncthreads();
                uint64_t *vb = bitmap + varoff[v];
                for (int64_t it = it0; it < it1; it++) foot_item(J, it, vb, l, 64, DevOr{});
            }
            __syncthreads();
            if (l == 0) signal(&vdone[2 * v]);
            continue;
        }
        tk -= C;
        if (tk < S) {  // fill segment
            const int64_t le = upper(send, ns, tk);
            const int64_t v = slist[le];
            int64_t local = tk - (le ? send[le - 1] : 0);
            const Prog &P = prog[v];
            int al = 0;
            while (P.arrcum[al] <= local) al++;
            local -= al ? P.arrcum[al - 1] : 0;
            if (l == 0) wait_for(&vdone[2 * v], P.chunks);
            __syncthreads();
            fill_segment(P, al, local, bitmap + varoff[v], foot + v * MAXARR * 2, l);
            __syncthreads();
            if (l == 0) signal(&vdone[2 * v + 1]);
            continue;
        }
        tk -= S;
        {  // finish variant dlist[tk]
            const int i = dlist[tk];
            const Prog &P = prog[i];
            if (l == 0) {
                wait_for(&vdone[2 * (int64_t)i], P.chunks);
                wait_for(&vdone[2 * (int64_t)i + 1], P.segs);
            }
            __syncthreads();
            if (l < MAXARR) {
                Fs[l] = foot[((int64_t)i * MAXARR + l) * 2];
                Fills[l] = foot[((int64_t)i * MAXARR + l) * 2 + 1];
            }
            __syncthreads();
            const int s2 = finalize_block(P, jobres + (int64_t)i * MAXJOB, Fs, Fills, PM_OK, fin,
                                          counts ? &counts[i] : nullptr, model, has_model,
                                          pred ? &pred[i] : nullptr);
            if (l == 0) status[i] = s2;
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- host ---
int launch_batch(Arena &ar, const Sched &sc, int nv, const pm_variant *d_var,
                 pm_counts *d_counts, const pm_model *model, double *d_pred,
                 int32_t *d_status, hipStream_t s, int n_cu, hipEvent_t *ev, int nmark) {
    int st = launch_expand(ar, sc, nv, d_var, d_counts, model, d_pred, d_status, s, ev, nmark);
    if (st) return st;
    return launch_rest(ar, sc, nv, d_counts, model, d_pred, d_status, s, n_cu, ev, nmark);
}

int launch_expand(Arena &ar, const Sched &sc, int nv, const pm_variant *d_var, pm_counts *d_counts,
                  const pm_model *model, double *d_pred, int32_t *d_status, hipStream_t s,
                  hipEvent_t *ev, int nmark) {
    if (nv <= 0) return PM_OK;
    pm_model m{};
    int has = 0;
    if (model) {
        m = *model;
        has = 1;
    }
    int64_t *meta = ar.meta + META_WORDS * ar.parity;
    int64_t *meta_next = ar.meta + META_WORDS * (ar.parity ^ 1);
    ar.parity ^= 1;
    const HandOn h{meta, meta_next, ar.varoff, ar.vdone, ar.clist, ar.slist, ar.dlist, ar.cend,
                   ar.send, (int64_t)ar.bitmap_words, (int64_t)ar.cap};
    // profiling events are taken by the dispatch itself (no extra packets
    // on the stream): start and end of the kernel
    hipEvent_t e0 = ev && nmark > 0 ? ev[0] : nullptr, e1 = ev && nmark > 1 ? ev[1] : nullptr;
    if (nv <= FUSED_MAX_NV)
        hipExtLaunchKernelGGL(k_fused, dim3(nv), dim3(FUSED_THREADS), 0, s, e0, e1, 0, nv, d_var,
                              ar.prog, ar.jobs, d_status, ar.jobres, ar.foot, h, d_counts, m,
                              has, d_pred, sc.fused_items);
    else
        hipExtLaunchKernelGGL(k_build, dim3(nv), dim3(64), 0, s, e0, e1, 0, nv, d_var, ar.prog,
                              ar.jobs, d_status, ar.jobres, ar.foot, h, d_counts, m, has, d_pred,
                              sc.inblock_items);
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}

int launch_rest(Arena &ar, const Sched &sc, int nv, pm_counts *d_counts, const pm_model *model,
                double *d_pred, int32_t *d_status, hipStream_t s, int n_cu, hipEvent_t *ev,
                int nmark) {
    if (nv <= 0) return PM_OK;
    const int grid = n_cu * sc.tail_wgs_per_cu;
    pm_model m{};
    int has = 0;
    if (model) {
        m = *model;
        has = 1;
    }
    int64_t *meta = ar.meta + META_WORDS * (ar.parity ^ 1);  // the last expansion's
    // one-wavefront work-groups: 4 x tail_wgs_per_cu per CU; events (taken
    // by the dispatch) at its start and end
    hipEvent_t e2 = ev && nmark > 2 ? ev[2] : nullptr, e3 = ev && nmark > 3 ? ev[3] : nullptr;
    hipExtLaunchKernelGGL(k_tail, dim3(4 * grid), dim3(64), 0, s, e2, e3, 0, (const Prog *)ar.prog,
                          (const Job *)ar.jobs, (const int32_t *)ar.clist,
                          (const int64_t *)ar.cend, (const int32_t *)ar.slist,
                          (const int64_t *)ar.send, (const int32_t *)ar.dlist,
                          (const int64_t *)ar.varoff, ar.bitmap, ar.jobres, ar.foot, ar.vdone,
                          d_status, d_counts, m, has, d_pred, meta, (int64_t)ar.cap,
                          (int64_t)ar.bitmap_words);
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}

size_t arena_bytes_per_variant() {
    return sizeof(Prog) + sizeof(Job) * MAXJOB +
           sizeof(int64_t) * (1 + 2 + 2 + MAXJOB + 2 * MAXARR) + sizeof(int32_t) * 3;
}

// ------------------------------------------------------- host execution ---
struct HostOr {
    void operator()(uint64_t *p, uint64_t m) const { *p |= m; }
};

int count_host(const pm_variant &v, pm_counts *out, int64_t *foot_out, bool sequential) {
    std::vector<Prog> P(1);
    std::vector<Job> J(MAXJOB);
    Prog &p = P[0];
    int st = sequential ? build_prog(v, &p, J.data()) : build_prog_slots(v, &p, J.data());
    for (int i = 0; i < PM_NCOUNT; i++) out->c[i] = 0;
    if (st != PM_OK) return st;
    std::vector<uint64_t> bm((size_t)p.bitmap_words + 1, 0);
    int64_t jobres[MAXJOB] = {0};
    int64_t F[MAXARR] = {0}, Fill[MAXARR] = {0};
    for (int j = 0; j < p.njob; j++) {
        if (p.jkind[j] == JOB_COUNT) {
            for (int64_t it = 0; it < J[j].items; it++) jobres[j] += count_item(J[j], it);
        } else if (p.jkind[j] == JOB_FOOT) {
            for (int64_t it = 0; it < J[j].items; it++) foot_item(J[j], it, bm.data(), 0, 1, HostOr{});
        }
    }
    for (int a = 0; a < p.narr; a++) {
        const ArrInfo &A = p.arr[a];
        if (!A.w || !A.words) continue;
        const uint64_t *f = bm.data() + A.f_off, *b = bm.data() + A.b_off;
        int64_t carry = -1;
        for (int64_t k = 0; k < A.words; k++) {
            uint64_t d = dilate_word(b[k], A.w) | carry_mask(carry, A.w, k);
            F[a] += __builtin_popcountll(f[k]);
            Fill[a] += __builtin_popcountll(f[k] | d);
            if (b[k]) carry = last_bit(b[k], k);
        }
    }
    if (foot_out)
        for (int a = 0; a < MAXARR; a++) {
            foot_out[2 * a] = F[a] + (a < p.narr ? p.arr[a].fixF : 0);
            foot_out[2 * a + 1] = Fill[a] + (a < p.narr ? p.arr[a].fixFill : 0);
        }
    return finalize(p, jobres, F, Fill, out->c);
}

}  // namespace pm
