// Kernel-variant descriptors and the per-variant parts of the counter.
//
// A variant (pm_variant) is expanded into a program: a list of statements,
// each an instruction of the kernel with
//   - a box domain over up to MAXVAR loop variables (group ids, local ids,
//     loop counters), each ranging over [0, ext),
//   - affine guards (sum c_v x_v + k >= 0) that restrict the domain,
//   - the global accesses it performs, each with an affine flat element
//     index (the index map I_j of Sec. 3.2, Alg. 2),
//   - per-instance tallies: LDS accesses, flops by kind/dtype, barriers.
// The count of every property is sum over statements of |domain| times the
// statement's tally (Sec. 3.2, Alg. 1, Eq. opcount).
//
// |domain| is computed without visiting every point:
//   * variables in no guard multiply the count by their extent;
//   * guarded variables split into connected components (variables linked
//     by a common guard); the count is the product of component counts;
//   * two variables a, b fuse into one of extent ext_a*ext_b when every
//     affine form of the component has coef_b == coef_a*ext_a;
//   * a one-variable component (or two that fuse) is an interval, counted
//     in closed form; larger components become jobs that enumerate all
//     variables but one and intersect the guards for the last (inner) one.
// Footprints (Alg. 2) of arrays with a lane stride >= 2 are sized in closed
// form when they are equally spaced runs, else marked in bitmaps by
// footprint jobs over the same fused domains.
//
// Everything here is __host__ __device__ (the expansion and finalize
// kernels run it on the GPU, and a host entry point runs it for unit tests)
// except LaneAff, the affine forms spread over a wavefront's lanes, which
// only the device's descriptor layout uses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm.h"

#define PM_HD __host__ __device__ inline

namespace pm {

constexpr int MAXVAR = 8;
constexpr int MAXGUARD = 4;  // the most any family needs (stencil halo, convolution tile)
constexpr int MAXACC = 5;    // per statement: the most any family needs (4 loads + 1 store)
constexpr int MAXACC_ALL = 12;  // per program (the stencil has 8)
constexpr int MAXSTMT = 10;  // the largest family (the stencil) has 9 statements
constexpr int MAXARR = 6;
constexpr int MAXJOB = 24;
constexpr int MAXCOMP = 4;
constexpr int NCLS = 15;

// count-vector layout (see pm.h)
constexpr int C_GACC = 0;
constexpr int C_LDS = 90;
constexpr int C_FLOP = 96;
constexpr int C_BARWI = 108;
constexpr int C_BARWG = 109;
constexpr int C_WG = 110;
constexpr int C_WI = 111;
// LDS accesses again, split by bank-stride bin: [dir][size][bin]
constexpr int NLBIN = 7;
constexpr int C_LDSB = 112;
static_assert(C_LDSB + 2 * 3 * NLBIN == PM_NCOUNT, "count-vector layout");

// Bank-stride bin of an LDS access whose address moves `words` 4-byte
// words when the lane index grows by one (Sec. 6.2: binning the stride of
// local memory access): 0 for a broadcast (stride 0), else 1 + the number
// of factors 2 in the stride, at most 6 -- odd strides (1), 2 x odd, ...,
// multiples of 32 (6).  With power-of-two bank counts the lanes of a
// wavefront that share a bank grow with that power of two.
PM_HD int lds_bin(int64_t words) {
    if (words == 0) return 0;
    const uint64_t w = (uint64_t)(words < 0 ? -words : words);
    const int v2 = __builtin_ctzll(w);
    return 1 + (v2 < NLBIN - 2 ? v2 : NLBIN - 2);
}
// An LDS access site of a statement: per instance `count` accesses of
// direction dir and size index z whose address moves `stride` words per
// lane, packed as count | bin << 16 | dir << 19 | z << 20 (0: no site).
constexpr int MAXLSITE = 4;
PM_HD uint32_t lsite_pack(int dir, int z, int bin, int count) {
    return (uint32_t)count | (uint32_t)bin << 16 | (uint32_t)dir << 19 | (uint32_t)z << 20;
}

enum { K_ADD = 0, K_MUL, K_DIV, K_EXP, K_SPEC, K_FMA };
enum { D_LD = 0, D_ST = 1 };
enum { JOB_NONE = 0, JOB_COUNT = 1, JOB_FOOT = 2 };

// inner points handled by one footprint work item
constexpr int64_t SEG_CONTIG = 16384;
constexpr int64_t SEG_STRIDED = 1024;
// bitmap words per fill segment (one wavefront of the chip-wide kernel)
constexpr int64_t SEG_WORDS = 4096;
// work items per chunk taken from the queue by one wavefront
constexpr int64_t CHUNK_COUNT = 2048;
constexpr int64_t CHUNK_FOOT = 4;

struct Aff {
    int64_t c[MAXVAR];
    int64_t k;
};

PM_HD Aff aff(int64_t k) {
    Aff a;
    for (int i = 0; i < MAXVAR; i++) a.c[i] = 0;
    a.k = k;
    return a;
}
PM_HD Aff av(Aff a, int v, int64_t coef) {
    a.c[v] += coef;
    return a;
}

struct GAcc {
    int32_t arr, dir, elem, vec;
    Aff idx;
};

struct Stmt {
    int32_t nvar, lane, nguard, nacc;
    uint64_t gmask;  // bits 8q..8q+7: variables with a non-zero coefficient in guard q
    int64_t ext[MAXVAR];
    Aff guard[MAXGUARD];
    int32_t acc0;  // its accesses are Prog::acc[acc0, acc0 + nacc)
    int32_t lds[2][3];
    uint32_t lsite[MAXLSITE];  // the same LDS accesses by site (lsite_pack)
    int32_t flop[6][2];
    int32_t bar;
    int32_t ncomp;
    int32_t comp_job[MAXCOMP];
    int64_t fixed;  // product of free extents and closed-form components
};

struct ArrInfo {
    int64_t cells;
    int64_t words;  // bitmap words (0: no footprint needed)
    int64_t f_off;  // word offset of F inside the variant's bitmap region
    int64_t b_off;  // word offset of B (cells of strided accesses); == f_off if same
    int64_t w;      // fill width of strided accesses: stride * vec cells
    int64_t segs;   // fill-pass segments (0: interval mode or no footprint)
    int64_t fixF, fixFill;  // interval mode: |F| and |Fill| in closed form
};

struct Prog {
    int32_t status, nstmt, narr, njob;
    // kind of the job in each slot (JOB_*): kept with the program so that a
    // variant counted where it was expanded never reads or clears slots in
    // the (slow) job memory it does not use
    int8_t jkind[MAXJOB];
    // the fast job buffer still holding the job of each slot (-1: the job
    // is only in its slot), when the expansion keeps jobs in its buffers
    int8_t jtmp[MAXJOB];
    int32_t wg_size;
    uint32_t flags;            // the variant's PM_FLAG_*
    int64_t n_wg;
    int64_t bitmap_words;
    int64_t chunks;            // work chunks of all jobs
    int64_t segs;              // fill segments of all bitmap arrays
    int64_t jobcum[MAXJOB];    // inclusive prefix of job chunks
    int64_t arrcum[MAXARR];    // inclusive prefix of array fill segments
    ArrInfo arr[MAXARR];
    int32_t nacc_all, pad;
    GAcc acc[MAXACC_ALL];      // global accesses of all statements, in order
    Stmt st[MAXSTMT];
};

// Access q of statement s.
PM_HD const GAcc &stmt_acc(const Prog &p, const Stmt &s, int q) { return p.acc[s.acc0 + q]; }

struct Job {
    int32_t kind, nv, ng, arr;
    int32_t vec, mark_b, pad0, pad1;
    int64_t ext[MAXVAR];                 // var 0 is the inner variable
    // affine forms, constant last: rows [0, ng) are the guards (>= 0), row
    // ng is the footprint index map (zero for count jobs)
    int64_t f[MAXGUARD + 1][MAXVAR + 1];
    int64_t seg, nseg, outer, items, chunk_items, chunks;
    int64_t f_off, b_off;            // bitmap word offsets (variant-relative)
    int64_t words;                   // words of each of this array's bitmaps
    int64_t w;                       // interval mode: fill width of a strided access, else 0
    // footprint jobs: interval-mode test and sizes, taken when the job is built
    int64_t ivF, ivFill;
    int32_t ivok, ivst;
};

// ------------------------------------------------------------- helpers ---
// Out of line: the rare 64-bit division stays out of the expansion
// kernels' hot code (which must fit the instruction cache).
#define PM_COLD __host__ __device__ __attribute__((noinline)) inline
PM_COLD int64_t div64_slow(int64_t a, int64_t b) { return a / b; }

PM_HD bool mul_ovf(int64_t a, int64_t b, int64_t *r) {
    // both factors within 32 bits (the usual case): the product fits
    if ((uint64_t)a + 0x80000000ull < 0x100000000ull &&
        (uint64_t)b + 0x80000000ull < 0x100000000ull) {
        *r = a * b;
        return false;
    }
    return __builtin_mul_overflow(a, b, r);
}
PM_HD bool add_ovf(int64_t a, int64_t b, int64_t *r) {
    return __builtin_add_overflow(a, b, r);
}
// a / b rounded toward zero (b != 0); the 32-bit divide when both fit,
// which is far shorter than the 64-bit sequence on the GPU.
PM_HD int64_t tdiv(int64_t a, int64_t b) {
    if (a == (int32_t)a && b == (int32_t)b && b != -1) return (int32_t)a / (int32_t)b;
    return div64_slow(a, b);
}
PM_HD int64_t cdiv(int64_t a, int64_t b) { return tdiv(a + b - 1, b); }
PM_HD int64_t tmod(int64_t a, int64_t b) { return a - tdiv(a, b) * b; }  // a % b
// floor(a / b) and ceil(a / b) for b > 0, any sign of a
PM_HD int64_t fdiv(int64_t a, int64_t b) {
    const int64_t q = tdiv(a, b);
    return (q * b != a && a < 0) ? q - 1 : q;
}
PM_HD int64_t ceil_div(int64_t a, int64_t b) {
    const int64_t q = tdiv(a, b);
    return (q * b != a && a > 0) ? q + 1 : q;
}
PM_HD int64_t iabs(int64_t a) { return a < 0 ? -a : a; }
PM_HD int size_index(int bytes) {
    return bytes == 4 ? 0 : bytes == 8 ? 1 : bytes == 16 ? 2 : -1;
}
PM_HD bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

// -------------------------------------------------------------- builder ---
// Affine forms while a descriptor is built.  RowAff: a whole form per
// thread (the host, or one device lane).  LaneAff (device): a wavefront
// holds one form, coefficient x in lane x and the constant in lane MAXVAR,
// so an update is one instruction and storing a row one store by nine
// lanes; every lane of the wavefront must run the builder together, with
// the same arguments.
struct RowAff {
    using V = Aff;
    static PM_HD V mk(int64_t k) { return aff(k); }
    static PM_HD V add(V a, int x, int64_t c) {
        a.c[x] += c;
        return a;
    }
    static PM_HD V add_k(V a, int64_t d) {
        a.k += d;
        return a;
    }
    static PM_HD V neg(V a) {
        for (int i = 0; i < MAXVAR; i++) a.c[i] = -a.c[i];
        a.k = -a.k;
        return a;
    }
    static PM_HD int64_t coef(const V &a, int x) { return a.c[x]; }
    static PM_HD uint64_t vars(const V &a) {  // bit x: coefficient x non-zero
        uint64_t m = 0;
        for (int x = 0; x < MAXVAR; x++)
            if (a.c[x]) m |= 1ull << x;
        return m;
    }
    static PM_HD void put(Aff *dst, const V &a) { *dst = a; }
    // a new statement: every field zero, the extents 1, its lane variable
    // and first access
    static PM_HD void stmt_init(Stmt *s, int lane_var, int a0) {
        for (size_t i = 0; i < sizeof(Stmt) / 8; i++) ((int64_t *)s)[i] = 0;
        for (int i = 0; i < MAXVAR; i++) s->ext[i] = 1;
        s->lane = lane_var;
        s->acc0 = a0;
    }
    // a statement's extents as a form (coefficient x: variable x's extent),
    // and their store with the statement's first ng guard rows
    static PM_HD V ones() {
        Aff a = aff(0);
        for (int i = 0; i < MAXVAR; i++) a.c[i] = 1;
        return a;
    }
    static PM_HD V set(V a, int x, int64_t v) {
        a.c[x] = v;
        return a;
    }
    static PM_HD void put_rows(Stmt *s, int nv, int ln, int ng, int na, uint64_t gm, const V &ext,
                               const V &g0, const V &g1, const V &g2, const V &g3) {
        s->nvar = nv;
        s->lane = ln;
        s->nguard = ng;
        s->nacc = na;
        s->gmask = gm;
        for (int x = 0; x < MAXVAR; x++) s->ext[x] = ext.c[x];
        const V *g[4] = {&g0, &g1, &g2, &g3};
        for (int q = 0; q < ng; q++) s->guard[q] = *g[q];
    }
    // a global access: its header and index map
    static PM_HD void put_acc(GAcc *g, const V &idx, int arr, int dir, int elem, int vec) {
        g->arr = arr;
        g->dir = dir;
        g->elem = elem;
        g->vec = vec;
        g->idx = idx;
    }
    template <class F>
    static PM_HD void each(int n, F f) {  // f(i) for i < n
        for (int i = 0; i < n; i++) f(i);
    }
    template <class F>
    static PM_HD void one(F f) {  // scalar stores
        f();
    }
};

struct LaneAff {
    struct V {
        int64_t v;
    };
    static __device__ int lane() { return (int)(threadIdx.x & 63); }
    static __device__ V mk(int64_t k) { return V{lane() == MAXVAR ? k : 0}; }
    static __device__ V add(V a, int x, int64_t c) { return V{a.v + (lane() == x ? c : 0)}; }
    static __device__ V add_k(V a, int64_t d) { return V{a.v + (lane() == MAXVAR ? d : 0)}; }
    static __device__ V neg(V a) { return V{-a.v}; }
    static __device__ int64_t coef(const V &a, int x) {
        const uint64_t u = (uint64_t)a.v;
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, x);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), x);
        return (int64_t)(((uint64_t)hi << 32) | lo);
    }
    static __device__ uint64_t vars(const V &a) {
        return __ballot(lane() < MAXVAR && a.v != 0) & ((1ull << MAXVAR) - 1);
    }
    static __device__ void put(Aff *dst, const V &a) {
        if (lane() <= MAXVAR) ((int64_t *)dst)[lane()] = a.v;  // c[0..MAXVAR), then k
    }
    // the same two as RowAff's, each one store by the lanes together: word
    // i of the statement by lane i (zero, 1 for the extents, the lane
    // variable and acc0 in their half-words); the index map by lanes
    // 0..MAXVAR as put() and the header's two words by the next two lanes
    static __device__ void stmt_init(Stmt *s, int lane_var, int a0) {
        constexpr int W = sizeof(Stmt) / 8, E0 = offsetof(Stmt, ext) / 8;
        constexpr int A0 = offsetof(Stmt, acc0) / 8;
        const int i = lane();
        if (i < W) {
            uint64_t v = i >= E0 && i < E0 + MAXVAR ? 1 : 0;
            v = i == 0 ? (uint64_t)(uint32_t)lane_var << 32 : v;  // nvar 0, lane
            v = i == A0 ? (uint64_t)(uint32_t)a0 : v;              // acc0, lds[0][0] 0
            ((uint64_t *)s)[i] = v;
        }
    }
    static __device__ V ones() { return V{1}; }
    static __device__ V set(V a, int x, int64_t v) { return V{lane() == x ? v : a.v}; }
    // lanes 0..MAXVAR together: the statement's first three words (its
    // counts and guard mask; lanes 0 and 1 the first two, the others the
    // third, equal values to one address), the extents (lane x: variable x's; lane MAXVAR: guard row
    // 0's constant, or 0 for a statement with no guard, whose zero rows
    // stay zero), then each guard row as put()
    static __device__ void put_rows(Stmt *s, int nv, int ln, int ng, int na, uint64_t gm,
                                    const V &ext, const V &g0, const V &g1, const V &g2,
                                    const V &g3) {
        const int i = lane();
        if (i <= MAXVAR) {
            const int w = i < 2 ? i : 2;
            const uint64_t hw = w == 0 ? (uint64_t)(uint32_t)ln << 32 | (uint32_t)nv
                              : w == 1 ? (uint64_t)(uint32_t)na << 32 | (uint32_t)ng : gm;
            ((uint64_t *)s)[w] = hw;
            int64_t *row = (int64_t *)&s->guard[0];
            *(i < MAXVAR ? &s->ext[i] : row + MAXVAR) = i < MAXVAR ? ext.v : ng > 0 ? g0.v : 0;
            if (ng > 0) row[i] = g0.v;
            if (ng > 1) row[(MAXVAR + 1) + i] = g1.v;
            if (ng > 2) row[2 * (MAXVAR + 1) + i] = g2.v;
            if (ng > 3) row[3 * (MAXVAR + 1) + i] = g3.v;
        }
    }
    static __device__ void put_acc(GAcc *g, const V &idx, int arr, int dir, int elem, int vec) {
        const int i = lane();
        if (i <= MAXVAR + 2) {
            const uint64_t h0 = (uint64_t)(uint32_t)dir << 32 | (uint32_t)arr;
            const uint64_t h1 = (uint64_t)(uint32_t)vec << 32 | (uint32_t)elem;
            const uint64_t v = i <= MAXVAR ? (uint64_t)idx.v : i == MAXVAR + 1 ? h0 : h1;
            uint64_t *dst = i <= MAXVAR ? (uint64_t *)&g->idx + i : (uint64_t *)g + (i - MAXVAR - 1);
            *dst = v;
        }
    }
    template <class F>
    static __device__ void each(int n, F f) {  // f(i) for i < n (n <= 64), lane i
        if (lane() < n) f(lane());
    }
    template <class F>
    static __device__ void one(F f) {  // scalar stores: by one lane, not 64 to one address
        if (lane() == 0) f();
    }
};
static_assert(offsetof(Aff, k) == MAXVAR * sizeof(int64_t), "row layout: c then k");
static_assert(offsetof(Stmt, nvar) == 0 && offsetof(Stmt, lane) == 4 &&
              offsetof(Stmt, acc0) % 8 == 0 && offsetof(Stmt, lds) == offsetof(Stmt, acc0) + 4 &&
              offsetof(Stmt, ext) % 8 == 0, "statement words that stmt_init writes");
static_assert(offsetof(GAcc, arr) == 0 && offsetof(GAcc, dir) == 4 && offsetof(GAcc, elem) == 8 &&
              offsetof(GAcc, vec) == 12 && offsetof(GAcc, idx) == 16, "access header: two words");
static_assert(sizeof(Stmt) % 8 == 0 && sizeof(Stmt) / 8 <= 64, "a statement is cleared one word per lane");
static_assert(MAXGUARD == 4 && sizeof(Aff) == (MAXVAR + 1) * 8, "put_rows: four guard rows of MAXVAR + 1 words");
static_assert(offsetof(Stmt, nguard) == 8 && offsetof(Stmt, nacc) == 12 && offsetof(Stmt, gmask) == 16,
              "put_rows: counts and guard mask in words 1 and 2");
static_assert(MAXJOB <= 64 && MAXVAR < 64, "LaneAff::each covers one wavefront");

template <class AP>
struct BT {
    using V = typename AP::V;
    Prog *p;
    // counts of the statement being built, kept in registers so that the
    // variable and guard indices of a builder are compile-time constants.
    // Builders fill one statement at a time: additions go to the latest.
    Stmt *cur = nullptr;
    int nvar = 0, nguard = 0, nacc = 0, lane = 0, nls = 0;
    // the program's statement, access and array counts and the current
    // statement's guard variable mask, also kept here (the program starts
    // empty); flush() stores the statement's once it is complete and the
    // program's at the end
    int nstmt = 0, nacc_all = 0, narr = 0;
    uint64_t gmask = 0;
    bool werr = false;  // an access with no whole lane stride, or two widths on one array
    // the current statement's LDS access counts by direction and size
    // (index dir * 3 + size) and the arrays' fill widths, kept here too, so
    // that lds() and acc() store without reading LDS back; a select chain
    // keeps them in scalar registers whatever the index
    int32_t lc0 = 0, lc1 = 0, lc2 = 0, lc3 = 0, lc4 = 0, lc5 = 0;
    int64_t aw0 = 0, aw1 = 0, aw2 = 0, aw3 = 0, aw4 = 0, aw5 = 0;
    // the current statement's extents and guard rows, stored by flush()
    // with one store each instead of one per declaration
    V extv = AP::ones(), g0 = AP::mk(0), g1 = AP::mk(0), g2 = AP::mk(0), g3 = AP::mk(0);
    PM_HD void set_guard(int q, const V &a) {
        g0 = q == 0 ? a : g0, g1 = q == 1 ? a : g1, g2 = q == 2 ? a : g2, g3 = q == 3 ? a : g3;
    }
    static_assert(MAXARR == 6, "one width register per array");
    PM_HD int64_t width(int a) const {
        return a == 0 ? aw0 : a == 1 ? aw1 : a == 2 ? aw2 : a == 3 ? aw3 : a == 4 ? aw4 : aw5;
    }
    PM_HD void set_width(int a, int64_t w) {
        aw0 = a == 0 ? w : aw0, aw1 = a == 1 ? w : aw1, aw2 = a == 2 ? w : aw2;
        aw3 = a == 3 ? w : aw3, aw4 = a == 4 ? w : aw4, aw5 = a == 5 ? w : aw5;
    }
    PM_HD int32_t add_lds(int k, int32_t count) {  // returns the new total of slot k
        const int32_t t = count + (k == 0 ? lc0 : k == 1 ? lc1 : k == 2 ? lc2
                                   : k == 3 ? lc3 : k == 4 ? lc4 : lc5);
        lc0 = k == 0 ? t : lc0, lc1 = k == 1 ? t : lc1, lc2 = k == 2 ? t : lc2;
        lc3 = k == 3 ? t : lc3, lc4 = k == 4 ? t : lc4, lc5 = k == 5 ? t : lc5;
        return t;
    }
    PM_HD void fail(int st) {
        if (p->status == PM_OK) p->status = st;
    }
    // store what is kept in registers: the current statement's counts,
    // guard mask, extents and guard rows when it starts the next statement,
    // and with `last` (the caller, when the family's builder has returned)
    // also the program's counts
    PM_HD void flush(bool last = false) {
        Stmt *s = cur;
        const int ns = nstmt, naa = nacc_all, nar = narr;
        Prog *pp = p;
        if (s) AP::put_rows(s, nvar, lane, nguard, nacc, gmask, extv, g0, g1, g2, g3);
        if (last)
            AP::one([=] {
                pp->nstmt = ns;
                pp->nacc_all = naa;
                pp->narr = nar;
            });
    }
    PM_HD Stmt *stmt(int lane_var) {
        flush();
        nvar = nguard = nacc = nls = 0;
        lc0 = lc1 = lc2 = lc3 = lc4 = lc5 = 0;
        extv = AP::ones();
        g0 = g1 = g2 = g3 = AP::mk(0);
        gmask = 0;
        lane = lane_var;
        cur = nullptr;
        if (nstmt >= MAXSTMT) {
            fail(PM_EINVAL);
            return nullptr;
        }
        Stmt *s = &p->st[nstmt++];
        cur = s;
        AP::stmt_init(s, lane_var, nacc_all);
        return s;
    }
    // declare variables in order; returns their ids 0..  (The id does not
    // depend on the extent, so it stays a compile-time constant; a failed
    // declaration marks the program invalid.)
    PM_HD int var(Stmt *s, int64_t ext) {
        if (s != cur) fail(PM_EINVAL);
        if (nvar >= MAXVAR) {
            fail(PM_EINVAL);
            return MAXVAR - 1;
        }
        if (ext < 0) fail(PM_EINVAL);
        const int x = nvar;
        extv = AP::set(extv, x, ext);
        return nvar++;
    }
    // affine forms of this builder
    PM_HD V mk(int64_t k) const { return AP::mk(k); }
    PM_HD V av(V a, int x, int64_t c) const { return AP::add(a, x, c); }
    PM_HD void ge0(Stmt *s, V a) {  // a >= 0
        if (s != cur || nguard >= MAXGUARD) {
            fail(PM_EINVAL);
            return;
        }
        set_guard(nguard, a);
        gmask |= AP::vars(a) << (8 * nguard);
        ++nguard;
    }
    PM_HD void lt(Stmt *s, V a, int64_t b) {  // a < b  <=>  (b-1) - a >= 0
        ge0(s, AP::add_k(AP::neg(a), b - 1));
    }
    PM_HD void ge(Stmt *s, V a, int64_t b) {  // a >= b
        ge0(s, AP::add_k(a, -b));
    }
    PM_HD void eq(Stmt *s, V a, int64_t b) {
        ge(s, a, b);
        lt(s, a, b + 1);
    }
    PM_HD void acc(Stmt *s, int arr, int dir, int elem, int vec, V idx) {
        if (s != cur || nacc >= MAXACC || nacc_all >= MAXACC_ALL || arr >= narr) {
            fail(PM_EINVAL);
            return;
        }
        GAcc *g = &p->acc[nacc_all++];
        AP::put_acc(g, idx, arr, dir, elem, vec);
        ++nacc;
        // the array's fill width: lane stride (in accesses) times the width
        // of a strided (stride >= 2) access
        const int64_t cl = AP::coef(idx, lane);
        const int64_t d = cl < 0 ? -cl : cl;
        const int64_t st = vec == 1 ? d : vec == 2 ? ((d & 1) ? -1 : d >> 1)
                         : vec == 4 ? ((d & 3) ? -1 : d >> 2) : -1;
        if (st < 0 || size_index(elem * vec) < 0) {
            werr = true;
        } else if (st >= 2) {
            ArrInfo *A = &p->arr[arr];
            const int64_t w = st * vec, w0 = width(arr);
            if (w0 && w0 != w) {
                werr = true;
            } else {
                set_width(arr, w);
                AP::one([=] { A->w = w; });
            }
        }
    }
    // `count` LDS accesses of `bytes` bytes per instance whose element index
    // moves `stride` elements when the lane index grows by one
    PM_HD void lds(Stmt *s, int dir, int bytes, int64_t stride, int count) {
        const int z = size_index(bytes);
        if (s != cur || nls >= MAXLSITE || z < 0 || count <= 0 || count >= (1 << 16)) {
            fail(PM_EINVAL);
            return;
        }
        const uint32_t site = lsite_pack(dir, z, lds_bin(stride * bytes / 4), count);
        const int k = nls++;
        const int32_t tot = add_lds(dir * 3 + z, count);
        AP::one([=] {
            s->lds[dir][z] = tot;
            s->lsite[k] = site;
        });
    }
    PM_HD void array(int a, int64_t cells) {
        if (a >= MAXARR) {
            fail(PM_EINVAL);
            return;
        }
        ArrInfo *A = &p->arr[a];
        set_width(a, 0);
        AP::one([=] {
            A->cells = cells;
            A->words = 0;
            A->f_off = A->b_off = -1;
            A->w = 0;
            A->segs = 0;
            A->fixF = A->fixFill = 0;
        });
        if (a + 1 > narr) narr = a + 1;
    }
};

template <class BB>
PM_HD int64_t prod3(BB &b, int64_t x, int64_t y, int64_t z) {
    int64_t r;
    if (mul_ovf(x, y, &r) || mul_ovf(r, z, &r)) {
        b.fail(PM_EOVERFLOW);
        return 0;
    }
    return r;
}

// --- stream: global-memory accesses at a lane stride and group stride ---
template <class BB>
PM_HD void build_stream(BB &b, const pm_variant &v) {
    int64_t N = v.n[0], wg = v.wg[0], s = v.stride, gs = v.gstride,
            vec = v.vec, U = v.reps;
    int e = v.dtype == PM_F64 ? 8 : 4;
    int dt = v.dtype == PM_F64 ? 1 : 0;
    if (N <= 0 || wg <= 0 || wg > 1024 || tmod(N, wg) || s < 1 || gs < 1 ||
        U < 1 || !(vec == 1 || vec == 2 || vec == 4) || e * vec > 16 ||
        v.op > PM_STREAM_AXPBY) {
        b.fail(PM_EINVAL);
        return;
    }
    int64_t G = tdiv(N, wg);
    b.p->n_wg = G;
    b.p->wg_size = (int32_t)wg;
    if (v.op == PM_STREAM_FILLED) {
        // of every s cells the first c are read: c accesses at lane stride s
        const int64_t c = v.chains ? v.chains : s;
        if (s < 2 || s > 64 || c < 1 || c > s || c > MAXACC || vec != 1 || gs != 1) {
            b.fail(PM_EINVAL);
            return;
        }
        b.array(0, prod3(b, s, N, U));
        b.array(1, N);
        Stmt *S = b.stmt(1);
        if (!S) return;
        int g = b.var(S, G), l = b.var(S, wg), u = b.var(S, U);
        for (int q = 0; q < c; q++)
            b.acc(S, 0, D_LD, e, 1, b.av(b.av(b.av(b.mk(q), g, s * wg), l, s), u, s * G * wg));
        S->flop[K_ADD][dt] = (int32_t)c;  // c - 1 in the group's sum, 1 into the running sum
        Stmt *T = b.stmt(1);
        if (!T) return;
        g = b.var(T, G);
        l = b.var(T, wg);
        b.acc(T, 1, D_ST, e, 1, b.av(b.av(b.mk(0), g, wg), l, 1));
        return;
    }
    int64_t span = prod3(b, G * gs, wg * s, U * vec);
    int na = v.op == PM_STREAM_ADD4 ? 5 : v.op == PM_STREAM_AXPBY ? 3 :
             v.op == PM_STREAM_COPY ? 2 : 1;
    for (int a = 0; a < na; a++) b.array(a, span);
    Stmt *S = b.stmt(1);
    if (!S) return;
    int g = b.var(S, G), l = b.var(S, wg), u = b.var(S, U);
    auto x = b.av(b.av(b.av(b.mk(0), g, vec * gs * wg * s), l, vec * s), u, vec * G * gs * wg * s);
    switch (v.op) {
    case PM_STREAM_LOAD:  // summed in a register; the sentinel store never runs
        b.acc(S, 0, D_LD, e, (int)vec, x);
        S->flop[K_ADD][dt] = (int32_t)vec;
        break;
    case PM_STREAM_STORE:
        b.acc(S, 0, D_ST, e, (int)vec, x);
        break;
    case PM_STREAM_COPY:
        b.acc(S, 0, D_LD, e, (int)vec, x);
        b.acc(S, 1, D_ST, e, (int)vec, x);
        break;
    case PM_STREAM_AXPBY:  // out = alpha x + beta y
        b.acc(S, 0, D_LD, e, (int)vec, x);
        b.acc(S, 1, D_LD, e, (int)vec, x);
        b.acc(S, 2, D_ST, e, (int)vec, x);
        S->flop[K_MUL][dt] = (int32_t)(2 * vec);
        S->flop[K_ADD][dt] = (int32_t)vec;
        break;
    default:  // add4
        for (int a = 0; a < 4; a++) b.acc(S, a, D_LD, e, (int)vec, x);
        b.acc(S, 4, D_ST, e, (int)vec, x);
        S->flop[K_ADD][dt] = (int32_t)(3 * vec);
    }
}

// --- LDS: R accesses per work-item at bank stride b ---
template <class BB>
PM_HD void build_lds(BB &b, const pm_variant &v) {
    int64_t G = v.n[0], wg = v.wg[0], R = v.reps, W = v.words;
    if (G <= 0 || wg <= 0 || wg > 1024 || R < 0 || v.stride < 1 ||
        !pow2(W) || W > 16384 || tmod(W, wg) || v.op > PM_LDS_WRITE) {
        b.fail(PM_EINVAL);
        return;
    }
    b.p->n_wg = G;
    b.p->wg_size = (int32_t)wg;
    b.array(0, G * wg);
    Stmt *S = b.stmt(1);
    if (!S) return;
    int g = b.var(S, G), l = b.var(S, wg);
    b.acc(S, 0, D_ST, 4, 1, b.av(b.av(b.mk(0), g, wg), l, 1));
    S->bar = 1;
    if (v.op == PM_LDS_READ) b.lds(S, D_ST, 4, 1, (int)tdiv(W, wg));  // initialisation lds[c*wg + l]
    else b.lds(S, D_LD, 4, v.stride, 1);  // read-back lds[(l*b) mod W]
    Stmt *L = b.stmt(1);
    if (!L) return;
    b.var(L, G);
    b.var(L, wg);
    b.var(L, R);
    if (v.op == PM_LDS_READ) {
        b.lds(L, D_LD, 4, v.stride, 1);  // lds[(l*b + r) mod W]
        L->flop[K_ADD][0] = 1;
    } else {
        b.lds(L, D_ST, 4, v.stride, 1);
    }
}

// --- FMA / rsqrt chains: 1 load, F ops, 1 store per work-item ---
// kind 0: FMA, 1: rsqrt, 2: division, 3: exponential
template <class BB>
PM_HD void build_chain(BB &b, const pm_variant &v, int kind) {
    int64_t N = v.n[0], wg = v.wg[0], F = v.reps, K = v.chains;
    int e = v.dtype == PM_F64 ? 8 : 4;
    int dt = v.dtype == PM_F64 ? 1 : 0;
    bool rsq = kind == 1;
    bool kok = kind ? (K == 1 || K == 2 || K == 4 || K == 8)
                    : (K == 1 || K == 2 || K == 4 || K == 8 || K == 16);
    if (N <= 0 || wg <= 0 || wg > 1024 || tmod(N, wg) || !kok || F < 0 || tmod(F, K) ||
        F > (1 << 24) || (rsq && v.dtype != PM_F32) || (kind >= 2 && v.op > PM_ARITH_EXP)) {
        b.fail(PM_EINVAL);
        return;
    }
    b.p->n_wg = tdiv(N, wg);
    b.p->wg_size = (int32_t)wg;
    b.array(0, N);
    b.array(1, N);
    Stmt *S = b.stmt(1);
    if (!S) return;
    int g = b.var(S, tdiv(N, wg)), l = b.var(S, wg);
    auto i = b.av(b.av(b.mk(0), g, wg), l, 1);
    b.acc(S, 0, D_LD, e, 1, i);
    b.acc(S, 1, D_ST, e, 1, i);
    if (rsq) {  // y = rsqrt(y*y + d)
        S->flop[K_MUL][dt] = (int32_t)F;
        S->flop[K_ADD][dt] = (int32_t)(F + K - 1);
        S->flop[K_SPEC][dt] = (int32_t)F;
    } else if (kind == 2) {  // y = d / (y*y + 1)
        S->flop[K_MUL][dt] = (int32_t)F;
        S->flop[K_ADD][dt] = (int32_t)(F + K - 1);
        S->flop[K_DIV][dt] = (int32_t)F;
    } else if (kind == 3) {  // y = exp(-(y*y)); the negation is not counted
        S->flop[K_MUL][dt] = (int32_t)F;
        S->flop[K_EXP][dt] = (int32_t)F;
        S->flop[K_ADD][dt] = (int32_t)(K - 1);
    } else {
        S->flop[K_FMA][dt] = (int32_t)F;
        S->flop[K_ADD][dt] = (int32_t)(K - 1);
    }
}

template <class BB>
PM_HD void build_barrier(BB &b, const pm_variant &v) {
    int64_t G = v.n[0], wg = v.wg[0], Bn = v.reps;
    if (G <= 0 || wg <= 0 || wg > 1024 || Bn < 0 || Bn > (1 << 20)) {
        b.fail(PM_EINVAL);
        return;
    }
    b.p->n_wg = G;
    b.p->wg_size = (int32_t)wg;
    b.array(0, G * wg);
    Stmt *S = b.stmt(1);
    if (!S) return;
    int g = b.var(S, G), l = b.var(S, wg);
    S->bar = (int32_t)Bn;
    b.acc(S, 0, D_ST, 4, 1, b.av(b.av(b.mk(0), g, wg), l, 1));
}

template <class BB>
PM_HD void build_empty(BB &b, const pm_variant &v) {
    int64_t n = v.n[0], wx = v.wg[0], wy = v.wg[1] ? v.wg[1] : 1;
    if (n <= 0 || wx <= 0 || wy <= 0 || wx * wy > 1024) {
        b.fail(PM_EINVAL);
        return;
    }
    b.p->n_wg = prod3(b, cdiv(n, wx), cdiv(n, wy), 1);
    b.p->wg_size = (int32_t)(wx * wy);
}

PM_HD bool tile_ok(int T) { return T == 8 || T == 16 || T == 32; }

// --- matmul: C[n,l] = A[n,m] B[m,l], T x T work-groups ---
template <class BB>
PM_HD void build_matmul(BB &b, const pm_variant &v) {
    int64_t n = v.n[0], m = v.n[1], L = v.n[2], T = v.tile;
    if (n <= 0 || m <= 0 || L <= 0 || !tile_ok((int)T) || v.dtype != PM_F32 ||
        v.op > PM_MATMUL_NAIVE || n > (1 << 24) || m > (1 << 24) || L > (1 << 24)) {
        b.fail(PM_EINVAL);
        return;
    }
    int64_t GX = cdiv(L, T), GY = cdiv(n, T), KT = cdiv(m, T);
    b.p->n_wg = GX * GY;
    b.p->wg_size = (int32_t)(T * T);
    b.array(0, n * m);
    b.array(1, m * L);
    b.array(2, n * L);
    // variables: 0 gy, 1 gx, 2 ly, 3 lx, then loop counters
    auto head = [&](Stmt *S) {
        b.var(S, GY);
        b.var(S, GX);
        b.var(S, T);
        b.var(S, T);
    };
    // Statements with guards are written over the fused indices their
    // guards test (row r = gy*T + ly, column c = gx*T + lx, and the k
    // offsets kt*T + lx or kt*T + ly of the tiles): the same points, each
    // guard on one variable; the lane variable is the index whose least
    // significant digit is lx
    const auto v0 = b.av(b.mk(0), 0, 1), v1 = b.av(b.mk(0), 1, 1), v2 = b.av(b.mk(0), 2, 1);
    if (v.op == PM_MATMUL_TILED) {
        Stmt *S = b.stmt(2);  // A tile element -> LDS: A[r][kt*T + lx]
        if (!S) return;
        b.var(S, GY * T);  // 0 r
        b.var(S, GX);      // 1 gx
        b.var(S, KT * T);  // 2 kt*T + lx
        b.lt(S, v0, n);
        b.lt(S, v2, m);
        b.acc(S, 0, D_LD, 4, 1, b.av(b.av(b.mk(0), 0, m), 2, 1));
        Stmt *Sb = b.stmt(2);  // B tile element -> LDS: B[kt*T + ly][c]
        if (!Sb) return;
        b.var(Sb, GY);      // 0 gy
        b.var(Sb, KT * T);  // 1 kt*T + ly
        b.var(Sb, GX * T);  // 2 c
        b.lt(Sb, v1, m);
        b.lt(Sb, v2, L);
        b.acc(Sb, 1, D_LD, 4, 1, b.av(b.av(b.mk(0), 1, L), 2, 1));
        Stmt *Sl = b.stmt(3);  // LDS stores (zero-padded outside) + 2 barriers
        if (!Sl) return;
        head(Sl);
        b.var(Sl, KT);
        b.lds(Sl, D_ST, 4, 1, 2);  // As[ly][lx], Bs[ly][lx]
        Sl->bar = 2;
        Stmt *Si = b.stmt(3);  // inner product step
        if (!Si) return;
        head(Si);
        b.var(Si, KT);
        b.var(Si, T);
        b.lds(Si, D_LD, 4, 0, 1);  // As[ly][k]: the same word for every lane
        b.lds(Si, D_LD, 4, 1, 1);  // Bs[k][lx]
        Si->flop[K_FMA][0] = 1;
    } else {
        Stmt *S = b.stmt(1);  // C[r][c] += A[r][k] * B[k][c]
        if (!S) return;
        b.var(S, GY * T);  // 0 r
        b.var(S, GX * T);  // 1 c
        b.var(S, m);       // 2 k
        b.lt(S, v0, n);
        b.lt(S, v1, L);
        b.acc(S, 0, D_LD, 4, 1, b.av(b.av(b.mk(0), 0, m), 2, 1));
        b.acc(S, 1, D_LD, 4, 1, b.av(b.av(b.mk(0), 2, L), 1, 1));
        S->flop[K_FMA][0] = 1;
    }
    Stmt *Sc = b.stmt(1);  // C[r][c]
    if (!Sc) return;
    b.var(Sc, GY * T);  // 0 r
    b.var(Sc, GX * T);  // 1 c
    b.lt(Sc, v0, n);
    b.lt(Sc, v1, L);
    b.acc(Sc, 2, D_ST, 4, 1, b.av(b.av(b.mk(0), 0, L), 1, 1));
}

// --- transpose: out[c][r] = in[r][c], n x n ---
template <class BB>
PM_HD void build_transpose(BB &b, const pm_variant &v) {
    int64_t n = v.n[0], T = v.tile;
    if (n <= 0 || n > (1 << 24) || !tile_ok((int)T) || v.dtype != PM_F32 ||
        v.op > PM_TRANSPOSE_NAIVE_RC) {
        b.fail(PM_EINVAL);
        return;
    }
    int64_t G = cdiv(n, T);
    b.p->n_wg = G * G;
    b.p->wg_size = (int32_t)(T * T);
    b.array(0, n * n);
    b.array(1, n * n);
    auto head = [&](Stmt *S) {
        b.var(S, G);  // 0 gy
        b.var(S, G);  // 1 gx
        b.var(S, T);  // 2 ly
        b.var(S, T);  // 3 lx
    };
    if (v.op == PM_TRANSPOSE_TILED) {
        // the guarded statements over the fused indices they test (the
        // lane variable holds lx as its least significant digit)
        const auto f0 = b.av(b.mk(0), 0, 1), f1 = b.av(b.mk(0), 1, 1);
        Stmt *S = b.stmt(1);  // in[r][c] -> tile[ly][lx]; r = gy*T + ly, c = gx*T + lx
        if (!S) return;
        b.var(S, G * T);
        b.var(S, G * T);
        b.lt(S, f0, n);
        b.lt(S, f1, n);
        b.acc(S, 0, D_LD, 4, 1, b.av(b.av(b.mk(0), 0, n), 1, 1));
        b.lds(S, D_ST, 4, 1, 1);  // tile[ly][lx], rows of T + 1
        Stmt *Sb = b.stmt(3);
        if (!Sb) return;
        head(Sb);
        Sb->bar = 1;
        Stmt *St = b.stmt(1);  // tile[lx][ly] -> out[r2][c2]; r2 = gx*T + ly, c2 = gy*T + lx
        if (!St) return;
        b.var(St, G * T);
        b.var(St, G * T);
        b.lt(St, f0, n);
        b.lt(St, f1, n);
        b.lds(St, D_LD, 4, T + 1, 1);  // tile[lx][ly]
        b.acc(St, 1, D_ST, 4, 1, b.av(b.av(b.mk(0), 0, n), 1, 1));
    } else {
        // one element per work-item and nothing shared within a group: the
        // domain written over the fused indices r = gy*T + ly and
        // c = gx*T + lx (extents G*T; c moves with the lane, by one per
        // lane like lx) -- the same points, index maps and lane strides
        Stmt *S = b.stmt(1);
        if (!S) return;
        b.var(S, G * T);  // 0 r
        b.var(S, G * T);  // 1 c
        const auto rf = b.av(b.mk(0), 0, 1), cf = b.av(b.mk(0), 1, 1);
        b.lt(S, rf, n);
        b.lt(S, cf, n);
        const auto rn_cf = b.av(b.av(b.mk(0), 0, n), 1, 1);  // r*n + c
        const auto cn_rf = b.av(b.av(b.mk(0), 1, n), 0, 1);  // c*n + r
        if (v.op == PM_TRANSPOSE_NAIVE_WC) {
            b.acc(S, 0, D_LD, 4, 1, cn_rf);
            b.acc(S, 1, D_ST, 4, 1, rn_cf);
        } else {
            b.acc(S, 0, D_LD, 4, 1, rn_cf);
            b.acc(S, 1, D_ST, 4, 1, cn_rf);
        }
    }
}

// --- 5-point stencil on an (n+2)^2 input with halo, T x T tiles in LDS ---
template <class BB>
PM_HD void build_stencil(BB &b, const pm_variant &v) {
    int64_t n = v.n[0], T = v.tile;
    if (n <= 0 || n > (1 << 24) || !tile_ok((int)T)) {
        b.fail(PM_EINVAL);
        return;
    }
    int e = v.dtype == PM_F64 ? 8 : 4;
    int dt = v.dtype == PM_F64 ? 1 : 0;
    int64_t G = cdiv(n, T), P = n + 2;
    b.p->n_wg = G * G;
    b.p->wg_size = (int32_t)(T * T);
    b.array(0, P * P);
    b.array(1, n * n);
    // Work-item (gy, gx, ly, lx) handles cell (i, j) = (gy*T + ly, gx*T + lx).
    // Each statement is written over the coarsest variables its guards allow:
    // (i, j) when it tests only i and j, (gy, ly, j) when it tests the row
    // within the tile, (i, gx, lx) when it tests the column within the tile.
    // These are the same points; the lane variable is lx, or j where lx is
    // part of it (j moves by one per lane, as lx does).
    auto ij = [&](Stmt *S) {  // 0 i, 1 j
        b.var(S, G * T);
        b.var(S, G * T);
    };
    auto rj = [&](Stmt *S) {  // 0 gy, 1 ly, 2 j
        b.var(S, G);
        b.var(S, T);
        b.var(S, G * T);
    };
    auto ic = [&](Stmt *S) {  // 0 i, 1 gx, 2 lx
        b.var(S, G * T);
        b.var(S, G);
        b.var(S, T);
    };
    // flat index of input cell (i + di, j + dj) in each variable set
    auto at_ij = [&](int64_t di, int64_t dj) {
        return b.av(b.av(b.mk(di * P + dj), 0, P), 1, 1);
    };
    auto at_rj = [&](int64_t di, int64_t dj) {
        return b.av(b.av(b.av(b.mk(di * P + dj), 0, T * P), 1, P), 2, 1);
    };
    auto at_ic = [&](int64_t di, int64_t dj) {
        return b.av(b.av(b.av(b.mk(di * P + dj), 0, P), 1, T), 2, 1);
    };
    const auto v0 = b.av(b.mk(0), 0, 1), v1 = b.av(b.mk(0), 1, 1), v2 = b.av(b.mk(0), 2, 1);
    // the last cell's tile and place in it: the partial last tile row
    // (column) is tile gl = (n-1) div T, its last row (column) rl = (n-1) mod T
    const int64_t gl = tdiv(n - 1, T), rl = n - 1 - gl * T, nt = tdiv(n, T);
    for (int q = 0; q < 7; q++) {
        // the tile and the halo rows: lane stride 1; the halo columns
        // (lx == 0, lx == T-1) are written at a fixed column.  The guards of
        // the last tile's halo are solved for the pinned variables:
        // ly == T-1 && gy*T + ly < n  <=>  ly == T-1 && gy < n div T, and
        // ly < T-1 && gy*T + ly == n-1  <=>  gy == gl && ly == rl < T-1
        // (that statement is written without gy); the same for columns
        Stmt *S = b.stmt(q == 0 || q == 3 ? 1 : 2);
        if (!S) return;
        if (q == 0) ij(S);
        else if (q <= 2) rj(S);
        else if (q == 3) {  // 0 ly, 1 j; gy = gl
            b.var(S, T);
            b.var(S, G * T);
        } else if (q <= 5) ic(S);
        else {  // 0 i, 1 gx (unused, extent 1), 2 lx; gx = gl
            b.var(S, G * T);
            b.var(S, 1);
            b.var(S, T);
        }
        b.lds(S, D_ST, e, q == 4 || q == 5 ? 0 : 1, 1);
        switch (q) {
        case 0:  // the tile, and the update of its cell (the same points)
            b.lt(S, v0, n), b.lt(S, v1, n);
            b.acc(S, 0, D_LD, e, 1, at_ij(1, 1));
            b.lds(S, D_LD, e, 1, 5);  // the point and its four neighbours, rows of T + 2
            S->flop[K_ADD][dt] = 4;  // N+S, +W, +E, + h^2 c^2
            S->flop[K_MUL][dt] = 3;  // c*c, h^2*(.), 0.25*(.)
            b.acc(S, 1, D_ST, e, 1, b.av(b.av(b.mk(0), 0, n), 1, 1));
            break;
        case 1:  // top halo row, loaded by ly == 0
            b.eq(S, v1, 0), b.lt(S, v2, n);
            b.acc(S, 0, D_LD, e, 1, at_rj(0, 1));
            break;
        case 2:  // bottom halo row of a full tile, loaded by ly == T-1
            b.eq(S, v1, T - 1), b.lt(S, v0, nt), b.lt(S, v2, n);
            b.acc(S, 0, D_LD, e, 1, at_rj(2, 1));
            break;
        case 3:  // bottom halo row of the last, partial tile row (none if it is full)
            if (rl < T - 1) b.eq(S, v0, rl);
            else b.lt(S, v0, 0);
            b.lt(S, v1, n);
            // cell (gl*T + ly + 2, j + 1)
            b.acc(S, 0, D_LD, e, 1, b.av(b.av(b.mk((gl * T + 2) * P + 1), 0, P), 1, 1));
            break;
        case 4:  // left halo column, loaded by lx == 0
            b.eq(S, v2, 0), b.lt(S, v0, n);
            b.acc(S, 0, D_LD, e, 1, at_ic(1, 0));
            break;
        case 5:  // right halo column of a full tile
            b.eq(S, v2, T - 1), b.lt(S, v0, n), b.lt(S, v1, nt);
            b.acc(S, 0, D_LD, e, 1, at_ic(1, 2));
            break;
        default:  // right halo column of the last, partial tile column (none if full)
            if (rl < T - 1) b.eq(S, v2, rl);
            else b.lt(S, v2, 0);
            b.lt(S, v0, n);
            // cell (i + 1, gl*T + lx + 2)
            b.acc(S, 0, D_LD, e, 1, b.av(b.av(b.mk(P + gl * T + 2), 0, P), 2, 1));
        }
    }
    Stmt *Sb = b.stmt(1);  // the barrier: every work-item, once
    if (!Sb) return;
    ij(Sb);
    Sb->bar = 1;
}

// --- all-pairs n-body: out[i] = sum_{j != i} rsqrt(|x_i - x_j|^2) ---
template <class BB>
PM_HD void build_nbody(BB &b, const pm_variant &v) {
    int64_t N = v.n[0], Gs = v.wg[0];
    if (N <= 0 || N > (1 << 26) || Gs < 64 || Gs > 1024 || Gs % 64 ||
        v.dtype != PM_F32) {
        b.fail(PM_EINVAL);
        return;
    }
    int64_t GB = cdiv(N, Gs);
    b.p->n_wg = GB;
    b.p->wg_size = (int32_t)Gs;
    b.array(0, 3 * N);
    b.array(1, N);
    Stmt *S = b.stmt(1);  // own position
    if (!S) return;
    int g = b.var(S, GB), l = b.var(S, Gs);
    auto i = b.av(b.av(b.mk(0), g, Gs), l, 1);
    b.lt(S, i, N);
    for (int c = 0; c < 3; c++)
        b.acc(S, 0, D_LD, 4, 1, b.av(b.av(b.mk(c), g, 3 * Gs), l, 3));
    Stmt *Sk = b.stmt(1);  // a block of positions -> LDS
    if (!Sk) return;
    g = b.var(Sk, GB), l = b.var(Sk, Gs);
    int jb = b.var(Sk, GB);
    b.lt(Sk, b.av(b.av(b.mk(0), jb, Gs), l, 1), N);
    for (int c = 0; c < 3; c++)
        b.acc(Sk, 0, D_LD, 4, 1, b.av(b.av(b.mk(c), jb, 3 * Gs), l, 3));
    b.lds(Sk, D_ST, 4, 1, 3);  // sh[c*G + l]
    Stmt *Sb = b.stmt(1);
    if (!Sb) return;
    b.var(Sb, GB), b.var(Sb, Gs), b.var(Sb, GB);
    Sb->bar = 2;
    Stmt *Sp = b.stmt(1);  // one pair
    if (!Sp) return;
    b.var(Sp, GB), b.var(Sp, Gs);
    jb = b.var(Sp, GB);
    int jj = b.var(Sp, Gs);
    b.lt(Sp, b.av(b.av(b.mk(0), jb, Gs), jj, 1), N);
    b.lds(Sp, D_LD, 4, 0, 3);  // sh[c*G + jj]: the same word for every lane
    Sp->flop[K_ADD][0] = 6;   // 3 differences, 2 adds in r^2, 1 into the block's partial
    Sp->flop[K_MUL][0] = 3;
    Sp->flop[K_SPEC][0] = 1;  // rsqrt; the self pair is masked by a select
    Stmt *Sa = b.stmt(1);  // the block's partial sum added to the total
    if (!Sa) return;
    b.var(Sa, GB), b.var(Sa, Gs), b.var(Sa, GB);
    Sa->flop[K_ADD][0] = 1;
    Stmt *So = b.stmt(1);
    if (!So) return;
    g = b.var(So, GB), l = b.var(So, Gs);
    b.lt(So, b.av(b.av(b.mk(0), g, Gs), l, 1), N);
    b.acc(So, 1, D_ST, 4, 1, b.av(b.av(b.mk(0), g, Gs), l, 1));
}

// --- convolution: three 7x7 filters over three RGB images ---
// Work-group (gx, gy, image zi, filter zj), T x T work-items; the filter and
// the (T+6)^2 x 3 image tile are staged through LDS.
template <class BB>
PM_HD void build_conv(BB &b, const pm_variant &v) {
    int64_t n = v.n[0], T = v.tile;
    if (n <= 0 || n > (1 << 20) || !(T == 8 || T == 16) || v.dtype != PM_F32) {
        b.fail(PM_EINVAL);
        return;
    }
    int64_t P = n + 6, G = cdiv(n, T), TT = T + 6;
    int64_t KF = cdiv(147, T * T), KA = cdiv(TT, T);
    b.p->n_wg = 9 * G * G;
    b.p->wg_size = (int32_t)(T * T);
    b.array(0, 3 * P * P * 3);
    b.array(1, 3 * 147);
    b.array(2, 9 * n * n);
    // variables: 0 gy, 1 gx, 2 zi, 3 zj, 4 ly, 5 lx, then loop counters
    auto head = [&](Stmt *S) {
        b.var(S, G);
        b.var(S, G);
        b.var(S, 3);
        b.var(S, 3);
        b.var(S, T);
        b.var(S, T);
    };
    Stmt *Sf = b.stmt(5);  // filter element t = k*T^2 + ly*T + lx -> LDS
    if (!Sf) return;
    head(Sf);
    int k = b.var(Sf, KF);
    auto t = b.av(b.av(b.av(b.mk(0), k, T * T), 4, T), 5, 1);
    b.lt(Sf, t, 147);
    b.acc(Sf, 1, D_LD, 4, 1, b.av(b.av(b.av(b.av(b.mk(0), 3, 147), k, T * T), 4, T), 5, 1));
    b.lds(Sf, D_ST, 4, 1, 1);  // fl[t]
    Stmt *Si = b.stmt(5);  // image tile cell (a*T + ly, b*T + lx), 3 channels
    if (!Si) return;
    head(Si);
    int a = b.var(Si, KA), bb = b.var(Si, KA);
    b.lt(Si, b.av(b.av(b.mk(0), a, T), 4, 1), TT);
    b.lt(Si, b.av(b.av(b.mk(0), bb, T), 5, 1), TT);
    b.lt(Si, b.av(b.av(b.av(b.mk(0), 0, T), a, T), 4, 1), P);
    b.lt(Si, b.av(b.av(b.av(b.mk(0), 1, T), bb, T), 5, 1), P);
    for (int c = 0; c < 3; c++)  // ((zi*P + X)*P + Y)*3 + c
        b.acc(Si, 0, D_LD, 4, 1,
              b.av(b.av(b.av(b.av(b.av(b.av(b.av(b.mk(c), 2, P * P * 3), 0, T * P * 3), a, T * P * 3),
                             4, P * 3), 1, T * 3), bb, T * 3), 5, 3));
    b.lds(Si, D_ST, 4, 3, 3);  // tile[r][q][c], channel fastest
    Stmt *Sb = b.stmt(5);
    if (!Sb) return;
    head(Sb);
    Sb->bar = 1;
    Stmt *Sm = b.stmt(5);  // one filter tap (u, v), three channels
    if (!Sm) return;
    head(Sm);
    b.var(Sm, 7);
    b.var(Sm, 7);
    auto x = b.av(b.av(b.mk(0), 0, T), 4, 1), y = b.av(b.av(b.mk(0), 1, T), 5, 1);
    b.lt(Sm, x, n);
    b.lt(Sm, y, n);
    b.lds(Sm, D_LD, 4, 3, 3);  // tile[ly + 6 - u][lx + 6 - v][c]
    b.lds(Sm, D_LD, 4, 0, 3);  // fl[(u*7 + v)*3 + c]: the same word for every lane
    Sm->flop[K_FMA][0] = 3;
    Stmt *So = b.stmt(5);
    if (!So) return;
    head(So);
    b.lt(So, x, n);
    b.lt(So, y, n);  // ((zi*3 + zj)*n + x)*n + y
    b.acc(So, 2, D_ST, 4, 1,
          b.av(b.av(b.av(b.av(b.av(b.av(b.mk(0), 2, 3 * n * n), 3, n * n), 0, T * n), 4, n), 1, T), 5, 1));
}

// ------------------------------------------------------ job preparation ---
// Fuse variables of a job whose affine forms treat (a, b) as one
// mixed-radix digit pair; returns the new variable count.
PM_HD int fuse(int nv, int64_t *ext, int nf, int64_t (*f)[MAXVAR + 1],
               bool *ovf) {
    // rows in which each variable appears: only variables with the same
    // rows can fuse, so the coefficients are compared for those pairs only
    uint32_t sig[MAXVAR];
    for (int x = 0; x < nv; x++) {
        uint32_t m = 0;
        for (int q = 0; q < nf; q++)
            if (f[q][x]) m |= 1u << q;
        sig[x] = m;
    }
    bool again = true;
    while (again && nv > 1) {
        again = false;
        for (int a = 0; a < nv && !again; a++)
            for (int bb = 0; bb < nv && !again; bb++) {
                if (a == bb || sig[a] != sig[bb]) continue;
                bool ok = true;
                for (uint32_t r = sig[a]; r && ok; r &= r - 1) {
                    const int q = __builtin_ctz(r);
                    int64_t want;
                    if (mul_ovf(f[q][a], ext[a], &want) || f[q][bb] != want) ok = false;
                }
                if (!ok) continue;
                int64_t e2;
                if (mul_ovf(ext[a], ext[bb], &e2)) {
                    *ovf = true;
                    return nv;
                }
                ext[a] = e2;
                // remove bb
                for (int t = bb; t < nv - 1; t++) {
                    ext[t] = ext[t + 1];
                    sig[t] = sig[t + 1];
                    for (int q = 0; q < nf; q++) f[q][t] = f[q][t + 1];
                }
                for (int q = 0; q < nf; q++) f[q][nv - 1] = 0;
                nv--;
                again = true;
            }
    }
    return nv;
}

// Narrow [lo, hi) of one variable by the guard c*x + k >= 0.
PM_HD void clip(int64_t c, int64_t k, int64_t &lo, int64_t &hi) {
    if (c == 1) {
        if (-k > lo) lo = -k;
    } else if (c == -1) {
        if (k + 1 < hi) hi = k + 1;
    } else if (c > 0) {
        const int64_t t = ceil_div(-k, c);
        if (t > lo) lo = t;
    } else if (c < 0) {
        const int64_t t = fdiv(k, -c) + 1;
        if (t < hi) hi = t;
    } else if (k < 0) {
        hi = lo;
    }
}

// Points of var x in [0, ext) under guards c*x + k >= 0 on a single
// variable (rows of g: coefficient in column 0, constant last).
PM_HD int64_t interval_count(int64_t ext, int ng, const int64_t (*g)[MAXVAR + 1]) {
    int64_t lo = 0, hi = ext;  // [lo, hi)
    for (int q = 0; q < ng; q++) clip(g[q][0], g[q][MAXVAR], lo, hi);
    return hi > lo ? hi - lo : 0;
}

// Closed-form count of a component of statement s with one variable, or
// with two that fuse (as fuse() would fuse them: (a, b) tried before
// (b, a)); guards `qs` (bit q: guard q touches the component).  Returns
// false when the component needs enumeration; *ovf on overflow.
// A two-variable component that does not fuse as a whole, but whose
// coupling guards (those on both variables) all act on one mixed-radix
// index x = major * E + minor (E the minor variable's extent) while every
// other guard bounds one of the two alone: the coupling guards bound x to
// an interval, the others bound the major digit and the minor digit
// (x mod E) to intervals, and the points are the x of the intersected
// interval whose remainder lies in the minor digit's interval -- a
// difference of two closed forms.  False when the component has no such
// form (it is then enumerated).
PM_HD bool mixed_radix_count(const int64_t *ca, const int64_t *cb, const int64_t *kq, uint32_t qs,
                             int64_t ea, int64_t eb, int64_t *cnt, bool *ovf) {
    bool a_major = true, b_major = true;  // orientations the coupling guards allow
    int64_t want;
#pragma unroll
    for (int q = 0; q < MAXGUARD; q++) {
        if (!((qs >> q) & 1) || !ca[q] || !cb[q]) continue;
        if (mul_ovf(cb[q], eb, &want) || ca[q] != want) a_major = false;
        if (mul_ovf(ca[q], ea, &want) || cb[q] != want) b_major = false;
    }
    if (!a_major && !b_major) return false;
    const int64_t *cM = a_major ? ca : cb, *cm = a_major ? cb : ca;
    const int64_t eM = a_major ? ea : eb, E = a_major ? eb : ea;
    int64_t X = 0;
    if (mul_ovf(eM, E, &X)) {
        *ovf = true;
        return true;
    }
    int64_t xlo = 0, xhi = X, mlo = 0, mhi = eM, nlo = 0, nhi = E;
#pragma unroll
    for (int q = 0; q < MAXGUARD; q++) {
        if (!((qs >> q) & 1)) continue;
        if (cM[q] && cm[q]) clip(cm[q], kq[q], xlo, xhi);  // cm * x + k >= 0
        else if (cM[q]) clip(cM[q], kq[q], mlo, mhi);
        else clip(cm[q], kq[q], nlo, nhi);
    }
    if (xhi <= xlo || mhi <= mlo || nhi <= nlo) {
        *cnt = 0;
        return true;
    }
    const int64_t x0 = xlo > mlo * E ? xlo : mlo * E;  // 0 <= mlo < mhi <= eM: no overflow
    const int64_t x1 = xhi < mhi * E ? xhi : mhi * E;
    if (x1 <= x0) {
        *cnt = 0;
        return true;
    }
    const int64_t w = nhi - nlo;
    // points x in [0, y) with x mod E in [nlo, nhi)
    auto below = [&](int64_t y) {
        const int64_t qy = tdiv(y, E), r = y - qy * E - nlo;
        return qy * w + (r < 0 ? 0 : r > w ? w : r);
    };
    *cnt = below(x1) - below(x0);
    return true;
}

PM_HD bool small_component(const Stmt &s, uint32_t M, uint32_t qs, int64_t *cnt, bool *ovf) {
    const int a = __builtin_ctz(M);
    const uint32_t rest = M & (M - 1);
    if (rest & (rest - 1)) return false;  // three or more variables
    const int b = rest ? __builtin_ctz(rest) : a;
    // both variables' coefficients and the constant of every guard row,
    // read at once (rows outside qs take no part)
    int64_t ca[MAXGUARD], cb[MAXGUARD], kq[MAXGUARD];
#pragma unroll
    for (int q = 0; q < MAXGUARD; q++) {
        ca[q] = s.guard[q].c[a];
        cb[q] = s.guard[q].c[b];
        kq[q] = s.guard[q].k;
    }
    int64_t ext = s.ext[a], lo = 0, hi;
    bool use_b = false;
    if (rest) {
        const int64_t ea = ext, eb = s.ext[b];
        // (x, y) fuses when every form has c_y == c_x * ext_x (both zero, or
        // both non-zero without overflow)
        bool fab = true, fba = true;
#pragma unroll
        for (int q = 0; q < MAXGUARD; q++) {
            if (!((qs >> q) & 1)) continue;
            int64_t want;
            if (ca[q] ? (!cb[q] || mul_ovf(ca[q], ea, &want) || cb[q] != want) : cb[q] != 0)
                fab = false;
            if (cb[q] ? (!ca[q] || mul_ovf(cb[q], eb, &want) || ca[q] != want) : ca[q] != 0)
                fba = false;
        }
        if (!fab && !fba) return mixed_radix_count(ca, cb, kq, qs, ea, eb, cnt, ovf);
        use_b = !fab;
        if (mul_ovf(ea, eb, &ext)) {
            *ovf = true;
            return true;
        }
    }
    hi = ext;
#pragma unroll
    for (int q = 0; q < MAXGUARD; q++)
        if ((qs >> q) & 1) clip(use_b ? cb[q] : ca[q], kq[q], lo, hi);
    *cnt = hi > lo ? hi - lo : 0;
    return true;
}

// Range [lo, hi) of the inner variable (var 0) for fixed outer values:
// r[q] is guard q evaluated on the outer variables.
PM_HD void inner_range(const Job &J, const int64_t *r, int64_t *lo_out,
                       int64_t *hi_out) {
    int64_t lo = 0, hi = J.ext[0];
    for (int q = 0; q < J.ng; q++) {
        int64_t a = J.f[q][0];
        if (a == 1) {
            if (-r[q] > lo) lo = -r[q];
        } else if (a == -1) {
            if (r[q] + 1 < hi) hi = r[q] + 1;
        } else if (a > 0) {
            int64_t t = ceil_div(-r[q], a);
            if (t > lo) lo = t;
        } else if (a < 0) {
            int64_t t = fdiv(r[q], -a) + 1;
            if (t < hi) hi = t;
        } else if (r[q] < 0) {
            hi = lo;
        }
    }
    *lo_out = lo;
    *hi_out = hi > lo ? hi : lo;
}

// Decompose outer point o (over vars 1..nv-1, var 1 fastest) and evaluate
// the guards and the index map on it.
// o is below the product of the outer extents, so the last variable's
// digit is what is left of o, with no division.
PM_HD void eval_outer(const Job &J, int64_t o, int64_t *r, int64_t *base) {
    for (int q = 0; q < J.ng; q++) r[q] = J.f[q][MAXVAR];
    int64_t b = J.f[J.ng][MAXVAR];
    for (int v = 1; v < J.nv; v++) {
        const int64_t e = J.ext[v];
        const int64_t q = v + 1 < J.nv ? tdiv(o, e) : 0, x = o - q * e;
        o = q;
        for (int q = 0; q < J.ng; q++) r[q] += J.f[q][v] * x;
        b += J.f[J.ng][v] * x;
    }
    *base = b;
}

// Lane stride of an access in units of the access size (-1: not whole).
PM_HD int64_t lane_stride(const Stmt &s, const GAcc &a) {
    const int64_t d = iabs(a.idx.c[s.lane]);
    switch (a.vec) {
    case 1: return d;
    case 2: return (d & 1) ? -1 : d >> 1;
    case 4: return (d & 3) ? -1 : d >> 2;
    default: return a.vec <= 0 || d % a.vec ? -1 : d / a.vec;
    }
}

// ---------------------------------------------------------- interval mode
// An array with a single footprint job whose fused domain has the inner
// variable t (index coefficient step > 0) and at most one outer variable x
// (coefficient c1 > 0), with no guard coupling t and x: every non-empty
// outer point covers the same inner range [lo, hi), so its cells are
// first(x) + step*t, t in [0, cnt), first(x) increasing in x, and the
// non-empty x form one interval.  Then
//   F    = union over x of its cells (a contiguous run when step <= vec,
//          else cnt disjoint accesses of vec cells),
//   Fill = union over x of [first, last cell + w)   (strided access), or F.
// The sizes then follow in closed form (ival).
// |F| and |Fill| of an array in interval mode.  Non-empty outer points x
// form an interval of nx values; each covers cnt accesses first(x) +
// step*t, first(x) = a0 + c1*x.  A run of accesses spans
// L = step*(cnt-1) + vec cells and, widened, Lf = L - 1 + w; nx runs spaced
// c1 apart cover L + (nx-1)*min(L, c1) cells when each run is contiguous
// (step <= vec) and nx*cnt*vec cells otherwise (runs are disjoint).
// One pass over the guards gives the inner range [lo, hi) (guards on t),
// the outer one [xlo, xhi) (guards on x) and whether a guard on no
// variable fails (the domain is empty).  *ok: the array qualifies (no
// guard couples t and x, runs do not interleave, widened accesses leave no
// gaps; an empty inner range qualifies); then F, Fill and the status (0, 0
// and PM_OK for an empty domain; PM_EOVERFLOW), else 0, 0 and PM_OK.
PM_HD int ival(const Job &J, bool *ok, int64_t *F, int64_t *Fill) {
    *ok = false;
    *F = *Fill = 0;
    if (J.nv > 2 || J.f[J.ng][0] <= 0) return PM_OK;
    if (J.nv == 2 && J.f[J.ng][1] <= 0) return PM_OK;
    int64_t lo = 0, hi = J.ext[0], xlo = 0, xhi = J.nv == 2 ? J.ext[1] : 1;
    bool cempty = false;
    for (int q = 0; q < J.ng; q++) {
        const int64_t a = J.f[q][0], b = J.nv == 2 ? J.f[q][1] : 0, r = J.f[q][MAXVAR];
        if (a && b) return PM_OK;
        const int64_t c = a ? a : b;
        int64_t &l = a ? lo : xlo, &h = a ? hi : xhi;
        if (!c) {
            if (r < 0) cempty = true;
        } else if (c > 0) {
            const int64_t t = ceil_div(-r, c);
            if (t > l) l = t;
        } else {
            const int64_t t = fdiv(r, -c) + 1;
            if (t < h) h = t;
        }
    }
    const int64_t cnt = hi > lo ? hi - lo : 0, step = J.f[J.ng][0], vec = J.vec;
    if (cnt != 0) {
        if (step > vec && J.nv == 2 && J.f[J.ng][1] < step * (cnt - 1) + vec) return PM_OK;
        if (J.w && step >= vec + J.w) return PM_OK;
    }
    *ok = true;
    const int64_t nx = xhi - xlo;
    if (cempty || cnt <= 0 || nx <= 0) return PM_OK;
    const int64_t c1 = J.nv == 2 ? J.f[J.ng][1] : 0;
    int64_t L, Lf, t;
    bool ovf = mul_ovf(step, cnt - 1, &L) || add_ovf(L, vec, &L);
    if (step <= vec) {
        ovf |= mul_ovf(nx - 1, L < c1 ? L : c1, &t) || add_ovf(L, t, F);
    } else {
        ovf |= mul_ovf(nx, cnt, &t) || mul_ovf(t, vec, F);
    }
    if (J.w) {
        ovf |= add_ovf(L, J.w - 1, &Lf);
        ovf |= mul_ovf(nx - 1, Lf < c1 ? Lf : c1, &t) || add_ovf(Lf, t, Fill);
    } else {
        *Fill = *F;
    }
    return ovf ? PM_EOVERFLOW : PM_OK;
}

// Copy of a finished job into its slot.
PM_HD void put_job(Job *dst, const Job &src) {
    const uint64_t *a = (const uint64_t *)&src;
    uint64_t *d = (uint64_t *)dst;
    for (size_t k = 0; k < sizeof(Job) / 8; k++) d[k] = a[k];
}

// The expansion of a variant into its program and jobs runs in three
// parts: build_head (statements, cleared job slots, fill widths),
// analyze_stmt for every statement (independent of each other), and
// build_tail (footprint modes, prefixes).  build_prog chains them.

// Statements of the variant's family, MAXJOB cleared job slots, and the
// fill width of every array with a strided access.  Returns the status.
template <class AP = RowAff>
PM_HD int build_head(const pm_variant &v, Prog *p, Job *jobs) {
    p->status = PM_OK;
    p->flags = v.flags;
    p->nstmt = p->narr = p->njob = 0;
    p->nacc_all = p->pad = 0;
    p->wg_size = 1;
    p->n_wg = 0;
    p->bitmap_words = 0;
    p->chunks = p->segs = 0;
    BT<AP> b{p};
    switch (v.family) {
    case PM_FAM_STREAM: build_stream(b, v); break;
    case PM_FAM_LDS: build_lds(b, v); break;
    case PM_FAM_FMA: build_chain(b, v, 0); break;
    case PM_FAM_RSQRT: build_chain(b, v, 1); break;
    case PM_FAM_ARITH: build_chain(b, v, v.op == PM_ARITH_EXP ? 3 : 2); break;
    case PM_FAM_CONV: build_conv(b, v); break;
    case PM_FAM_BARRIER: build_barrier(b, v); break;
    case PM_FAM_EMPTY: build_empty(b, v); break;
    case PM_FAM_MATMUL: build_matmul(b, v); break;
    case PM_FAM_TRANSPOSE: build_transpose(b, v); break;
    case PM_FAM_STENCIL: build_stencil(b, v); break;
    case PM_FAM_NBODY: build_nbody(b, v); break;
    default: b.fail(PM_EINVAL);
    }
    b.flush(true);
    AP::each(MAXJOB, [=](int j) {
        p->jkind[j] = JOB_NONE;
        p->jtmp[j] = -1;
    });
    // arrays needing footprints got their fill widths as accesses were added
    if (p->status == PM_OK && b.werr) b.fail(PM_EINVAL);
    return p->status;
}

// Counts of statement si (its fixed factor and components) and its jobs,
// numbered from `base`: a job number reaching `cap` returns `over`.  Jobs
// are assembled in the buffer temp() gives when the first one is made
// (fast memory next to a slow `jobs`), else (nullptr) in their slots, and
// copied to their slots -- except, when `keep` (the first of the buffers
// temp() hands out) is given, the statement's last job, which stays in its
// buffer (p->jtmp).  *made: jobs made.  Reads the program and writes only
// statement si and its job slots, so statements may be analysed
// concurrently.  Returns a status.
template <class TEMP>
PM_HD int analyze_stmt(Prog *p, int si, Job *jobs, TEMP temp, int base, int cap, int over,
                       int *made, const Job *keep = nullptr) {
    int nj = base;
    *made = 0;
    Job *jt = nullptr;
    bool asked = false;
    int prev = -1;  // slot whose job the buffer still holds (keep)
    // the buffer is about to take another job: its last one goes to its slot
    auto release = [&]() {
        if (jt && prev >= 0) {
            put_job(&jobs[prev], *jt);
            p->jtmp[prev] = -1;
            prev = -1;
        }
    };
    // job nj is complete in the buffer: keep it there, or copy it out
    auto settle = [&]() {
        if (!jt) return;
        if (keep) {
            p->jtmp[nj] = (int8_t)(jt - keep);
            prev = nj;
        } else {
            put_job(&jobs[nj], *jt);
        }
    };
    Stmt &s = p->st[si];
    s.ncomp = 0;
    const int nvar = s.nvar, ng = s.nguard;
    bool empty = false;
    // the statement's extents (undeclared ones are 1) and guard constants,
    // read at once (rows past nguard are not used)
    int64_t ext[MAXVAR], kq[MAXGUARD];
#pragma unroll
    for (int x = 0; x < MAXVAR; x++) ext[x] = s.ext[x];
#pragma unroll
    for (int q = 0; q < MAXGUARD; q++) kq[q] = s.guard[q].k;
#pragma unroll
    for (int x = 0; x < MAXVAR; x++)
        if (ext[x] == 0) empty = true;
    // variables of each guard (8 bits per guard) and of all guards
    const uint64_t gm = s.gmask;
    const uint32_t vmask = (1u << nvar) - 1;  // declared variables
    uint32_t guarded = 0;
#pragma unroll
    for (int q = 0; q < MAXGUARD; q++) {
        if (q >= ng) break;
        const uint32_t m = (uint32_t)(gm >> (8 * q)) & vmask;
        guarded |= m;
        if (!m && kq[q] < 0) empty = true;
    }
    if (empty) {
        s.fixed = 0;
        return PM_OK;
    }
    int64_t fixed = 1;
    bool fovf = false;
#pragma unroll
    for (int x = 0; x < MAXVAR; x++)
        if (x < nvar && !((guarded >> x) & 1) && mul_ovf(fixed, ext[x], &fixed)) fovf = true;
    if (fovf) return PM_EOVERFLOW;
    // one count per component: variables linked through common guards
    uint32_t done = 0;
    for (int root = 0; root < nvar; root++) {
        if (!((guarded >> root) & 1) || ((done >> root) & 1)) continue;
        uint32_t M = 1u << root;
        for (bool grow = true; grow;) {
            grow = false;
            for (int q = 0; q < ng; q++) {
                const uint32_t m = (uint32_t)(gm >> (8 * q)) & vmask;
                if ((m & M) && (m & ~M)) {
                    M |= m;
                    grow = true;
                }
            }
        }
        done |= M;
        uint32_t qs = 0;
        for (int q = 0; q < ng; q++)
            if ((gm >> (8 * q)) & M) qs |= 1u << q;
        int64_t c;
        bool ovf = false;
        // closed form, unless the variant asks for enumeration (cross-checks)
        if (!(p->flags & PM_FLAG_ENUMERATE) && small_component(s, M, qs, &c, &ovf)) {
            if (ovf || mul_ovf(fixed, c, &fixed)) return PM_EOVERFLOW;
            continue;
        }
        if (nj >= cap) return over;
        if (s.ncomp >= MAXCOMP) return PM_EINVAL;
        if (!asked) jt = temp(), asked = true;
        release();
        // the job, assembled in a fast buffer when one was given, else in
        // its slot: 1 made, 0 an interval (its count in c), < 0 a status
        auto count_job = [&](Job &J) __attribute__((always_inline)) -> int {
            J.kind = JOB_COUNT;
            J.nv = 0;
            J.ng = 0;
            J.arr = -1;
            J.vec = 1;
            J.mark_b = 0;
            // job column t: the component's t-th variable (increasing order)
            int xt[MAXVAR];
            const int ncol = __builtin_popcount(M);
            {
                uint32_t r = M;
#pragma unroll
                for (int t = 0; t < MAXVAR; t++) {
                    xt[t] = r ? __builtin_ctz(r) : 0;
                    r &= r - 1;
                }
            }
            J.nv = ncol;
#pragma unroll
            for (int t = 0; t < MAXVAR; t++)
                if (t < ncol) J.ext[t] = s.ext[xt[t]];
            for (uint32_t r = qs; r; r &= r - 1) {
                const int q = __builtin_ctz(r);
                int64_t row[MAXVAR];
#pragma unroll
                for (int t = 0; t < MAXVAR; t++) row[t] = t < ncol ? s.guard[q].c[xt[t]] : 0;
#pragma unroll
                for (int t = 0; t < MAXVAR; t++) J.f[J.ng][t] = row[t];
                J.f[J.ng][MAXVAR] = s.guard[q].k;
                J.ng++;
            }
            // two variables reach here only when small_component found that
            // they fuse in neither order, which is fuse()'s test on these rows
            // (or when enumeration is asked for: then they stay two)
            if (ncol > 2) J.nv = fuse(J.nv, J.ext, J.ng, J.f, &ovf);
            if (ovf) return PM_EOVERFLOW;
            if (J.nv == 1) {  // an interval: closed form, the slot is reused
                c = interval_count(J.ext[0], J.ng, J.f);
                return 0;
            }
            // inner variable: the largest extent
            int in = 0;
            for (int x = 1; x < J.nv; x++)
                if (J.ext[x] > J.ext[in]) in = x;
            if (in) {
                int64_t te = J.ext[0];
                J.ext[0] = J.ext[in];
                J.ext[in] = te;
                for (int q = 0; q < J.ng; q++) {
                    int64_t tg = J.f[q][0];
                    J.f[q][0] = J.f[q][in];
                    J.f[q][in] = tg;
                }
            }
            for (int t = 0; t <= MAXVAR; t++) J.f[J.ng][t] = 0;  // no index map
            J.outer = 1;
            for (int x = 1; x < J.nv; x++)
                if (mul_ovf(J.outer, J.ext[x], &J.outer)) return PM_EOVERFLOW;
            J.seg = J.ext[0];
            J.nseg = 1;
            J.items = J.outer;
            J.chunk_items = CHUNK_COUNT;
            J.chunks = cdiv(J.items, CHUNK_COUNT);
            J.f_off = J.b_off = 0;
            J.words = 0;
            J.w = 0;
            J.ivok = 0;
            return 1;
        };
        Job &Jc = jt ? *jt : jobs[nj];  // one copy of the builder for both memories
        const int rj = count_job(Jc);
        if (rj < 0) return rj;
        if (rj == 0) {
            if (mul_ovf(fixed, c, &fixed)) return PM_EOVERFLOW;
            continue;
        }
        settle();
        p->jkind[nj] = JOB_COUNT;
        s.comp_job[s.ncomp++] = nj++;
    }
    s.fixed = fixed;
    // footprint jobs for accesses to arrays with a strided access
    for (int q = 0; q < s.nacc; q++) {
        const GAcc &a = stmt_acc(*p, s, q);
        ArrInfo &A = p->arr[a.arr];
        if (!A.w) continue;
        if (nj >= cap) return over;
        if (!asked) jt = temp(), asked = true;
        release();
        // assembled like the count jobs: 1 made, < 0 a status
        auto foot_job = [&](Job &J) __attribute__((always_inline)) -> int {
            J.kind = JOB_FOOT;
            J.nv = 0;
            J.ng = 0;
            J.arr = a.arr;
            J.vec = a.vec;
            J.mark_b = lane_stride(s, a) >= 2;  // strided: its cells are widened
            J.f_off = J.b_off = -1;             // set with the array's mode below
            J.words = 0;
            J.w = J.mark_b ? A.w : 0;
            // variables: every guarded one and those of the index map, in
            // increasing order (job column t = the t-th of them)
            uint32_t Mf = guarded;
#pragma unroll
            for (int x = 0; x < MAXVAR; x++)
                if (a.idx.c[x]) Mf |= 1u << x;
            Mf &= vmask;
            int xt[MAXVAR];
            const int ncol = __builtin_popcount(Mf);
            {
                uint32_t r = Mf;
#pragma unroll
                for (int t = 0; t < MAXVAR; t++) {
                    xt[t] = r ? __builtin_ctz(r) : 0;
                    r &= r - 1;
                }
            }
            J.nv = ncol;
#pragma unroll
            for (int t = 0; t < MAXVAR; t++)
                if (t < ncol) J.ext[t] = s.ext[xt[t]];
            for (int g = 0; g < ng; g++) {
                int64_t row[MAXVAR];
#pragma unroll
                for (int t = 0; t < MAXVAR; t++) row[t] = t < ncol ? s.guard[g].c[xt[t]] : 0;
#pragma unroll
                for (int t = 0; t < MAXVAR; t++) J.f[J.ng][t] = row[t];
                J.f[J.ng][MAXVAR] = s.guard[g].k;
                J.ng++;
            }
            int64_t *ic = J.f[J.ng];  // the index map after the guards
            {
                int64_t row[MAXVAR];
#pragma unroll
                for (int t = 0; t < MAXVAR; t++) row[t] = t < ncol ? a.idx.c[xt[t]] : 0;
#pragma unroll
                for (int t = 0; t < MAXVAR; t++) ic[t] = row[t];
                ic[MAXVAR] = a.idx.k;
            }
            // fuse over guards and the index map together (two variables
            // can fuse only when they appear in the same rows)
            bool ovf = false;
            bool same_rows = J.nv > 2;
            if (J.nv == 2) {
                same_rows = true;
                for (int q = 0; q <= J.ng; q++)
                    if ((J.f[q][0] != 0) != (J.f[q][1] != 0)) same_rows = false;
            }
            if (same_rows) J.nv = fuse(J.nv, J.ext, J.ng + 1, J.f, &ovf);
            if (ovf) return PM_EOVERFLOW;
            if (J.nv == 0) {  // a single access point
                J.nv = 1;
                J.ext[0] = 1;
            }
            // inner variable: smallest non-zero index coefficient
            int in = -1;
            for (int x = 0; x < J.nv; x++) {
                if (!ic[x]) continue;
                if (in < 0 || iabs(ic[x]) < iabs(ic[in]) ||
                    (iabs(ic[x]) == iabs(ic[in]) && J.ext[x] > J.ext[in]))
                    in = x;
            }
            if (in < 0) in = 0;
            if (in) {
                int64_t te = J.ext[0];
                J.ext[0] = J.ext[in];
                J.ext[in] = te;
                for (int g = 0; g <= J.ng; g++) {
                    int64_t tg = J.f[g][0];
                    J.f[g][0] = J.f[g][in];
                    J.f[g][in] = tg;
                }
            }
            J.outer = 1;
            for (int x = 1; x < J.nv; x++)
                if (mul_ovf(J.outer, J.ext[x], &J.outer)) return PM_EOVERFLOW;
            J.seg = iabs(ic[0]) <= J.vec ? SEG_CONTIG : SEG_STRIDED;
            J.nseg = cdiv(J.ext[0], J.seg);
            if (mul_ovf(J.outer, J.nseg, &J.items)) return PM_EOVERFLOW;
            J.chunk_items = CHUNK_FOOT;
            J.chunks = cdiv(J.items, CHUNK_FOOT);
            bool ok;
            int64_t fF, fFill;
            const int ist = ival(J, &ok, &fF, &fFill);
            J.ivok = ok;
            J.ivst = ist;
            J.ivF = fF;
            J.ivFill = fFill;
            return 1;
        };
        Job &Jf = jt ? *jt : jobs[nj];
        const int rf = foot_job(Jf);
        if (rf < 0) return rf;
        settle();
        p->jkind[nj] = JOB_FOOT;
        nj++;
    }
    *made = nj - base;
    return PM_OK;
}

// Footprint mode of every strided array over job slots [0, nj), then the
// chunk and segment prefixes.  Returns the status.
// `prefix`: also the job-chunk and fill-segment prefixes (a caller that
// computes them itself, from the same values, passes false).
PM_HD int build_tail(const pm_variant &v, Prog *p, Job *jobs, int nj,
                     Job *keep = nullptr, bool prefix = true) {
    p->njob = nj;
    // slot j's job: in its buffer when the expansion kept it there
    auto JB = [&](int j) -> Job & { return keep && p->jtmp[j] >= 0 ? keep[p->jtmp[j]] : jobs[j]; };

    // Each strided array: interval mode when its footprint is a sequence of
    // equally spaced runs (ival: sizes in closed form), else bitmaps.
    int64_t off = 0;
    for (int ai = 0; ai < p->narr; ai++) {
        ArrInfo &A = p->arr[ai];
        if (!A.w) continue;
        int nfj = 0, fj = -1;
        for (int j = 0; j < nj; j++)
            if (p->jkind[j] == JOB_FOOT && JB(j).arr == ai) nfj++, fj = j;
        if (nfj == 1 && !(v.flags & PM_FLAG_BITMAP) && JB(fj).ivok) {
            Job &J = JB(fj);
            if (J.ivst != PM_OK) return p->status = PM_EOVERFLOW;
            A.fixF = J.ivF;
            A.fixFill = J.ivFill;
            J.kind = JOB_NONE;  // nothing left to enumerate
            p->jkind[fj] = JOB_NONE;
            J.items = J.chunks = 0;
            A.words = 0;
            A.segs = 0;
            continue;
        }
        bool mixed = false;  // a stride <= 1 access: widened cells kept apart
        for (int j = 0; j < nj; j++)
            if (p->jkind[j] == JOB_FOOT && JB(j).arr == ai && !JB(j).mark_b) mixed = true;
        A.words = (A.cells + A.w + 8 + 63) / 64 + 1;
        A.f_off = off;
        off += A.words;
        if (mixed) {
            A.b_off = off;
            off += A.words;
        } else {
            A.b_off = A.f_off;
        }
        A.segs = cdiv(A.words, SEG_WORDS);
        for (int j = 0; j < nj; j++) {
            if (p->jkind[j] != JOB_FOOT) continue;
            Job &J = JB(j);
            if (J.arr != ai) continue;
            J.f_off = A.f_off;
            J.b_off = J.mark_b ? A.b_off : -1;
            J.mark_b = J.mark_b && A.b_off != A.f_off;
            J.words = A.words;
        }
    }
    p->bitmap_words = off;
    if (!prefix) return p->status;
    int64_t cum = 0;
    for (int j = 0; j < MAXJOB; j++) {
        cum += j < nj && p->jkind[j] != JOB_NONE ? JB(j).chunks : 0;
        p->jobcum[j] = cum;
    }
    p->chunks = cum;
    cum = 0;
    for (int a = 0; a < MAXARR; a++) {
        cum += (a < p->narr && p->arr[a].w && p->arr[a].words) ? p->arr[a].segs : 0;
        p->arrcum[a] = cum;
    }
    p->segs = cum;
    return p->status;
}

// Expand a variant into its program and jobs.  `jobs` has MAXJOB slots.
// Each job is assembled in *jt when given (fast memory next to a slow
// `jobs`), else in its slot.  Returns the status; sets per-array bitmap
// needs and prog->bitmap_words.
PM_HD int build_prog(const pm_variant &v, Prog *p, Job *jobs, Job *jt = nullptr) {
    int st = build_head(v, p, jobs);
    if (st != PM_OK) return st;
    int nj = 0;
    for (int si = 0; si < p->nstmt; si++) {
        int k;
        st = analyze_stmt(p, si, jobs, [jt]() { return jt; }, nj, MAXJOB, PM_EINVAL, &k);
        if (st != PM_OK) return p->status = st;
        nj += k;
    }
    return build_tail(v, p, jobs, nj);
}

// The expansion with statements analysed independently: statement si
// gets job slots 2si and 2si+1.  After analyze_stmt(p, si, jobs, ., 2si,
// 2si+2, PM_SEQ, .) returned r[si] for every statement, build_slots_finish
// completes it: the first failing statement's status, or the tail over
// 2*nstmt slots; a statement that wanted more than two jobs sends the
// variant through build_prog instead (compact slots, same counts).
constexpr int PM_SEQ = 1000;  // internal: more than two jobs in a statement
static_assert(2 * MAXSTMT <= MAXJOB, "two job slots per statement");
PM_HD int build_slots_finish(const pm_variant &v, Prog *p, Job *jobs, Job *jt, const int *r) {
    const int ns = p->nstmt;
    for (int si = 0; si < ns; si++) {
        if (r[si] == PM_SEQ) return build_prog(v, p, jobs, jt);
        if (r[si] != PM_OK) return p->status = r[si];
    }
    return build_tail(v, p, jobs, 2 * ns);
}

// The sequential re-analysis build_slots_finish falls back to, on a
// program whose statements are already laid out (build_head ran): job
// slots compact from 0, each statement analysed in order with the same
// temp() as the per-statement pass (so both share one analyze_stmt).
template <class TEMP>
PM_HD int build_seq(const pm_variant &v, Prog *p, Job *jobs, TEMP temp) {
    for (int j = 0; j < MAXJOB; j++) {
        p->jkind[j] = JOB_NONE;
        p->jtmp[j] = -1;
    }
    int nj = 0;
    for (int si = 0; si < p->nstmt; si++) {
        int k;
        const int st = analyze_stmt(p, si, jobs, temp, nj, MAXJOB, PM_EINVAL, &k);
        if (st != PM_OK) return p->status = st;
        nj += k;
    }
    return build_tail(v, p, jobs, nj);
}

// build_slots_finish with the fallback through build_seq.
template <class TEMP>
PM_HD int build_slots_finish_seq(const pm_variant &v, Prog *p, Job *jobs, TEMP temp,
                                 const int *r, Job *keep, bool prefix = true) {
    const int ns = p->nstmt;
    for (int si = 0; si < ns; si++) {
        if (r[si] == PM_SEQ) return build_seq(v, p, jobs, temp);
        if (r[si] != PM_OK) return p->status = r[si];
    }
    return build_tail(v, p, jobs, 2 * ns, keep, prefix);
}

// Host form of the same: the statements one after another.
PM_HD int build_prog_slots(const pm_variant &v, Prog *p, Job *jobs) {
    int st = build_head(v, p, jobs);
    if (st != PM_OK) return st;
    int r[MAXSTMT];
    for (int si = 0; si < p->nstmt; si++) {
        int made;
        r[si] = analyze_stmt(p, si, jobs, []() { return (Job *)nullptr; }, 2 * si, 2 * si + 2,
                             PM_SEQ, &made);
    }
    return build_slots_finish(v, p, jobs, nullptr, r);
}

// --------------------------------------------------- footprint marking ---
// Marks of one footprint item: cells first + step*t, t in [0, cnt), each
// covering vec cells, OR-ed into bitmap bm.  Work is split over `nl`
// lanes; lane `ln` does its share.  ORfn(word_ptr, mask) performs the OR.
// Words outside [0, nwords) are never touched.
template <class ORF>
PM_HD void mark_run(uint64_t *bm, int64_t nwords, int64_t first, int64_t step,
                    int64_t cnt, int64_t vec, int ln, int nl, ORF orf) {
    if (cnt <= 0 || first < 0) return;
    auto orb = [&](int64_t w, uint64_t m) {
        if (w >= 0 && w < nwords) orf(bm + w, m);
    };
    if (step <= vec) {  // one contiguous range
        int64_t a = first, e = first + step * (cnt - 1) + vec;  // [a, e)
        int64_t w0 = a >> 6, w1 = (e - 1) >> 6;
        for (int64_t w = w0 + ln; w <= w1; w += nl) {
            uint64_t m = ~0ull;
            if (w == w0) m &= ~0ull << (a & 63);
            if (w == w1) m &= ~0ull >> (63 - ((e - 1) & 63));
            orb(w, m);
        }
    } else if (step <= 64) {  // several accesses per word: build word masks
        int64_t e = first + step * (cnt - 1) + vec;
        int64_t w0 = first >> 6, w1 = (e - 1) >> 6;
        for (int64_t w = w0 + ln; w <= w1; w += nl) {
            int64_t lo = w << 6, hi = lo + 64;
            int64_t t = lo - vec + 1 - first;
            t = t <= 0 ? 0 : ceil_div(t, step);
            uint64_t m = 0;
            for (; t < cnt; t++) {
                int64_t c = first + step * t;
                if (c >= hi) break;
                for (int64_t z = 0; z < vec; z++) {
                    int64_t cz = c + z;
                    if (cz >= lo && cz < hi) m |= 1ull << (cz - lo);
                }
            }
            if (m) orb(w, m);
        }
    } else {  // one access per word
        for (int64_t t = ln; t < cnt; t += nl) {
            int64_t c = first + step * t;
            for (int64_t z = 0; z < vec; z++) {
                int64_t cz = c + z;
                orb(cz >> 6, 1ull << (cz & 63));
            }
        }
    }
}

// Process footprint item `it` of job J (lane ln of nl cooperating lanes).
template <class ORF>
PM_HD void foot_item(const Job &J, int64_t it, uint64_t *vbase, int ln, int nl,
                     ORF orf) {
    const int64_t o = tdiv(it, J.nseg), sg = it - o * J.nseg;
    int64_t r[MAXGUARD], base, lo, hi;
    eval_outer(J, o, r, &base);
    inner_range(J, r, &lo, &hi);
    int64_t s0 = sg * J.seg, s1 = s0 + J.seg;
    if (lo < s0) lo = s0;
    if (hi > s1) hi = s1;
    if (hi <= lo) return;
    int64_t c0 = J.f[J.ng][0];
    int64_t first, step;
    if (c0 >= 0) {
        first = base + c0 * lo;
        step = c0;
    } else {
        first = base + c0 * (hi - 1);
        step = -c0;
    }
    int64_t cnt = hi - lo;
    if (step == 0) cnt = 1;
    mark_run(vbase + J.f_off, J.words, first, step, cnt, J.vec, ln, nl, orf);
    if (J.mark_b) mark_run(vbase + J.b_off, J.words, first, step, cnt, J.vec, ln, nl, orf);
}

// Count of count-job item `it` (one outer point).
PM_HD int64_t count_item(const Job &J, int64_t it) {
    int64_t r[MAXGUARD], base, lo, hi;
    eval_outer(J, it, r, &base);
    inner_range(J, r, &lo, &hi);
    return hi - lo;
}

// ------------------------------------------------------------ fill pass ---
// Dilation of the set bits of m by [0, w) inside one word.
PM_HD uint64_t dilate_word(uint64_t m, int64_t w) {
    int64_t ext = 1;
    while (ext < w && ext < 64) {
        int64_t sh = ext < w - ext ? ext : w - ext;
        m |= m << sh;
        ext += sh;
    }
    return m;
}
// Bits of word k covered by a run [last, last + w) that started before it.
PM_HD uint64_t carry_mask(int64_t last, int64_t w, int64_t k) {
    if (last < 0) return 0;
    int64_t n = last + w - (k << 6);
    if (n <= 0) return 0;
    if (n >= 64) return ~0ull;
    return (1ull << n) - 1;
}
PM_HD int64_t last_bit(uint64_t m, int64_t k) {
    return m ? (k << 6) + 63 - __builtin_clzll(m) : -1;
}

// ------------------------------------------------------------- finalize ---
PM_HD int class_index(int64_t s, int64_t F, int64_t Fill) {
    if (s == 0) return 0;
    if (s == 1) return 1;
    int64_t q = s < 4 ? s : 4;
    if (Fill <= 0) return s == 2 ? 2 : s == 3 ? 4 : s == 4 ? 7 : 11;
    int64_t k = cdiv(q * F, Fill);
    if (k < 1) k = 1;
    if (k > q) k = q;
    int base = s == 2 ? 2 : s == 3 ? 4 : s == 4 ? 7 : 11;
    return base + (int)(k - 1);
}

// The count vector is assembled from a list of contributions: statement
// `stmt` adds mult x (its number of executions) to slot `slot`.  Each
// statement has NENT candidate entries -- its global accesses, LDS accesses
// by direction and size, flops by kind and dtype, barriers -- of which only
// the non-zero ones enter the list.  The same helpers serve the host loop
// (finalize) and the 64-lane version on the device.
constexpr int NENT = MAXACC + 6 + 12 + 1 + MAXLSITE;
struct Contrib {
    int16_t slot, stmt;
    int32_t mult;
};

// Executions of statement si: its free extents and closed-form components
// (s.fixed) times the counts of its enumerated components.  False on
// overflow.
PM_HD bool stmt_count(const Prog &p, int si, const int64_t *jobres, int64_t *out) {
    const Stmt &s = p.st[si];
    int64_t cnt = s.fixed;
    bool ok = true;
    for (int q = 0; q < s.ncomp; q++)
        if (mul_ovf(cnt, jobres[s.comp_job[q]], &cnt)) ok = false;
    *out = cnt;
    return ok;
}

// Entry e (0 <= e < NENT) of statement si: true with *c set when present.
// A global access's slot follows from its size, direction and stride class
// (Sec. 2, classes from Alg. 2's footprints F and Fill of its array).
PM_HD bool contrib(const Prog &p, int si, int e, const int64_t *F, const int64_t *Fill,
                   Contrib *c) {
    const Stmt &s = p.st[si];
    c->stmt = (int16_t)si;
    if (e < MAXACC) {
        if (e >= s.nacc) return false;
        const GAcc &a = stmt_acc(p, s, e);
        const int64_t st = lane_stride(s, a);
        const int z = size_index(a.elem * a.vec);
        const int cl = class_index(st, F[a.arr] + p.arr[a.arr].fixF,
                                   Fill[a.arr] + p.arr[a.arr].fixFill);
        c->slot = (int16_t)(C_GACC + (a.dir * 3 + z) * NCLS + cl);
        c->mult = 1;
        return true;
    }
    e -= MAXACC;
    if (e < 6) {
        c->slot = (int16_t)(C_LDS + e);
        c->mult = s.lds[e / 3][e % 3];
    } else if (e < 18) {
        e -= 6;
        c->slot = (int16_t)(C_FLOP + e);
        c->mult = s.flop[e / 2][e % 2];
    } else if (e == 18) {
        c->slot = (int16_t)C_BARWI;
        c->mult = s.bar;
    } else {  // an LDS site, in its bank-stride bin
        const uint32_t w = s.lsite[e - 19];
        const int dir = (w >> 19) & 1, z = (w >> 20) & 3, bin = (w >> 16) & 7;
        c->slot = (int16_t)(C_LDSB + (dir * 3 + z) * NLBIN + bin);
        c->mult = (int32_t)(w & 0xffff);
    }
    return c->mult != 0;
}

// Value of count slot k from the contribution list; false on overflow.
// Slots without entries are 0; C_WG / C_WI come from the launch shape and
// C_BARWG from C_BARWI (set by the caller).
// Slot k of the count vector summed exactly (overflow-checked) over every
// statement's contributions.
PM_HD bool slot_sum(const Prog &p, int k, const int64_t *F, const int64_t *Fill,
                    const int64_t *sc, int64_t *out) {
    if (k == C_WG) {
        *out = p.n_wg;
        return true;
    }
    if (k == C_WI) return !mul_ovf(p.n_wg, (int64_t)p.wg_size, out);
    int64_t v = 0, t;
    bool ok = true;
    for (int si = 0; si < p.nstmt; si++)
        for (int e = 0; e < NENT; e++) {
            Contrib cc;
            if (!contrib(p, si, e, F, Fill, &cc) || cc.slot != k) continue;
            if (mul_ovf(sc[si], (int64_t)cc.mult, &t) || add_ovf(v, t, &v)) ok = false;
        }
    *out = v;
    return ok;
}
PM_HD int finalize(const Prog &p, const int64_t *jobres, const int64_t *F,
                   const int64_t *Fill, int64_t *c) {
    for (int i = 0; i < PM_NCOUNT; i++) c[i] = 0;
    if (p.status != PM_OK) return p.status;
    bool ok = true;
    int64_t sc[MAXSTMT];
    for (int si = 0; si < p.nstmt; si++)
        if (!stmt_count(p, si, jobres, &sc[si])) ok = false;
    for (int k = 0; k < PM_NCOUNT; k++)
        if (k != C_BARWG && !slot_sum(p, k, F, Fill, sc, &c[k])) ok = false;
    c[C_BARWG] = p.wg_size ? c[C_BARWI] / p.wg_size : 0;
    if (!ok) {
        for (int i = 0; i < PM_NCOUNT; i++) c[i] = 0;
        return PM_EOVERFLOW;
    }
    return PM_OK;
}

// ------------------------------------------------------------- features ---
PM_HD int nfeat(uint32_t proj) {
    return proj == PM_PROJ_P3 ? 3 : proj == PM_PROJ_P12 ? 12 : proj == PM_PROJ_FULL ? 154 :
           proj == PM_PROJ_EXT ? 157 : proj == PM_PROJ_BANK ? 193 : -1;
}
// PM_PROJ_BANK feature j: the 42 binned LDS counts in place of
// PM_PROJ_EXT's 6 (features 90..95); returns the PM_PROJ_EXT feature it
// equals, or -1 with *slot the count slot it reads.
PM_HD int bank_to_ext(int j, int *slot) {
    if (j < 90) return j;
    if (j < 90 + 42) {
        *slot = C_LDSB + (j - 90);
        return -1;
    }
    return j - 36;
}

PM_HD bool full_use_class(int cl) {  // '0', '1', '2/2', '3/3', '4/4'
    return cl == 0 || cl == 1 || cl == 3 || cl == 6 || cl == 10;
}

// Feature j of projection `proj` from count vector c.
PM_HD double feature_one(const int64_t *c, uint32_t proj, int j) {
    const double SZ[3] = {4, 8, 16};
    if (proj == PM_PROJ_BANK) {
        int slot = 0;
        j = bank_to_ext(j, &slot);
        if (j < 0) return (double)c[slot];
        proj = PM_PROJ_EXT;
    }
    if (proj == PM_PROJ_P3) {
        if (j == 0) {  // global bytes, every class and direction
            double gb = 0;
            for (int d = 0; d < 2; d++)
                for (int z = 0; z < 3; z++)
                    for (int cl = 0; cl < NCLS; cl++)
                        gb += SZ[z] * (double)c[C_GACC + (d * 3 + z) * NCLS + cl];
            return gb;
        }
        return j == 1 ? (double)c[C_FLOP + K_FMA * 2 + 0] : (double)c[C_WG];
    }
    if (proj == PM_PROJ_P12) {
        switch (j) {
        case 0: return 1.0;
        case 1: return (double)c[C_WG];
        case 2: return (double)c[C_BARWI];
        case 3:
        case 4: {
            const int d = j - 3;
            return (double)c[C_FLOP + K_ADD * 2 + d] + (double)c[C_FLOP + K_MUL * 2 + d] +
                   2.0 * (double)c[C_FLOP + K_FMA * 2 + d];
        }
        case 5: {
            double sp = 0;
            for (int d = 0; d < 2; d++)
                sp += (double)c[C_FLOP + K_SPEC * 2 + d] + (double)c[C_FLOP + K_DIV * 2 + d] +
                      (double)c[C_FLOP + K_EXP * 2 + d];
            return sp;
        }
        case 6: {
            double ldsb = 0;
            for (int d = 0; d < 2; d++)
                for (int z = 0; z < 3; z++) ldsb += SZ[z] * (double)c[C_LDS + d * 3 + z];
            return ldsb;
        }
        case 7: case 8: case 9: case 10: {  // full-use / partial-use bytes per direction
            const int d = (j - 7) & 1;
            const bool want_full = j < 9;
            double x = 0;
            for (int z = 0; z < 3; z++)
                for (int cl = 0; cl < NCLS; cl++)
                    if (full_use_class(cl) == want_full)
                        x += SZ[z] * (double)c[C_GACC + (d * 3 + z) * NCLS + cl];
            return x;
        }
        default: {  // min(unit-stride load bytes, unit-stride store bytes)
            double s1[2] = {0, 0};
            for (int d = 0; d < 2; d++)
                for (int z = 0; z < 3; z++) s1[d] += SZ[z] * (double)c[C_GACC + (d * 3 + z) * NCLS + 1];
            return s1[0] < s1[1] ? s1[0] : s1[1];
        }
        }
    }
    if (proj == PM_PROJ_EXT && j >= 154) {
        double ops = 0, gb = 0;
        for (int k = 0; k < 12; k++) ops += (double)c[C_FLOP + k];
        for (int d = 0; d < 2; d++)
            for (int z = 0; z < 3; z++)
                for (int cl = 0; cl < NCLS; cl++)
                    gb += SZ[z] * (double)c[C_GACC + (d * 3 + z) * NCLS + cl];
        const double wi = (double)(c[C_WI] < PM_RESIDENT_WI ? c[C_WI] : PM_RESIDENT_WI);
        if (j == 154) return wi > 0 ? ops / wi : 0.0;
        if (j == 155) return wi > 0 ? gb / wi : 0.0;
        return ops < gb ? ops : gb;
    }
    // PM_PROJ_FULL: every global class, LDS, flops (an FMA counts as one add
    // and one mul), barriers, work-groups, a constant, min(load, store) per
    // size and class
    if (j < 90) return (double)c[C_GACC + j];
    if (j < 96) return (double)c[C_LDS + j - 90];
    if (j < 106) {
        const int k = (j - 96) / 2, d = (j - 96) % 2;
        double x = (double)c[C_FLOP + k * 2 + d];
        if (k == K_ADD || k == K_MUL) x += (double)c[C_FLOP + K_FMA * 2 + d];
        return x;
    }
    if (j == 106) return (double)c[C_BARWI];
    if (j == 107) return (double)c[C_WG];
    if (j == 108) return 1.0;
    const int z = (j - 109) / NCLS, cl = (j - 109) % NCLS;
    const int64_t ld = c[C_GACC + (0 * 3 + z) * NCLS + cl];
    const int64_t st = c[C_GACC + (1 * 3 + z) * NCLS + cl];
    return (double)(ld < st ? ld : st);
}

PM_HD int features(const int64_t *c, uint32_t proj, double *f) {
    const int n = nfeat(proj);
    for (int j = 0; j < n; j++) f[j] = feature_one(c, proj, j);
    return n;
}

// T = sum_i alpha_i f_i.  The summation order is fixed so that every device
// path gives the same bits: 64 partial sums, partial l over features
// i = l, l+64, ... in increasing order, then combined pairwise at distances
// 32, 16, ..., 1 (the order of a 64-lane butterfly reduction).
PM_HD double predict_partial(const int64_t *c, const pm_model &m, int lane) {
    const int nf = nfeat(m.proj) < (int)m.nfeat ? nfeat(m.proj) : (int)m.nfeat;
    double t = 0.0;
    for (int i = lane; i < nf; i += 64) t += m.alpha[i] * feature_one(c, m.proj, i);
    return t;
}

PM_HD double predict(const int64_t *c, const pm_model &m) {
    double part[64];
    for (int l = 0; l < 64; l++) part[l] = predict_partial(c, m, l);
    for (int off = 32; off > 0; off >>= 1) {
        double nxt[64];
        for (int l = 0; l < 64; l++) nxt[l] = part[l] + part[l ^ off];
        for (int l = 0; l < 64; l++) part[l] = nxt[l];
    }
    return part[0];
}

}  // namespace pm
