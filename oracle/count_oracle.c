/*
 * Count oracle: simulated execution of every kernel family.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls
 * this file; only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (the paper's Sec. 2 properties, Sec. 3.2 Alg. 1 and 2):
 * each family is a loop nest that mirrors its kernel source work-item by
 * work-item.  Every global access, LDS access, floating point operation and
 * barrier a work-item would execute is emitted as an event and tallied, so
 * an instruction's count is the number of points of its (guarded) domain
 * that actually execute it (Alg. 1, Eq. opcount).
 *
 *   - global accesses are keyed by access size (4/8/16 bytes), direction
 *     and amortized stride fraction (Sec. 2.1);
 *   - the lane stride of a static access site is the change of its flat
 *     element index when local id 0 grows by one, divided by the elements
 *     per access; guards are ignored for this (the index map decides);
 *   - the utilization ratio is per array (Alg. 2): |F| / |Fill| where F is
 *     the set of touched cells and Fill adds, for every cell x touched by a
 *     site of stride s >= 2, the run [x, x + s*vec) (gaps between strided
 *     accesses filled in).  Classes: s=0 -> '0', s=1 -> '1', s>=2 ->
 *     'k/q' with q = min(s,4) and k = ceil(q * |F| / |Fill|) in exact
 *     integer arithmetic ('>4' bins for s>4);
 *   - LDS accesses by size and direction (Sec. 2.1, last par.), and again
 *     by bank-stride bin (Sec. 6.2, binning the stride of local memory
 *     access): the stride of an LDS site is the change of its element
 *     index when local id 0 grows by one (the unmasked affine index, guards
 *     ignored), in 4-byte words; bin 0 for stride 0, else 1 + the number of
 *     factors 2 in it, at most 6;
 *   - flops by kind (add/sub, mul, div, exp/pow, special, fma) and fp32 or
 *     fp64; integer and index arithmetic is not counted (Sec. 2.2);
 *   - barriers summed over all work-items (Sec. 2.3) and per work-group;
 *     work-groups and work-items launched (Sec. 2.4).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define O_NSZ 3
#define O_NCLS 15
#define O_NKIND 6
#define O_MAXSITE 16
#define O_MAXARR 8

/* output layout of this oracle (its own; the HIP library has another) */
#define O_GACC 0                      /* [dir][size][class] : 90 */
#define O_LDS (O_GACC + 2 * O_NSZ * O_NCLS) /* [dir][size] : 6 */
#define O_FLOP (O_LDS + 2 * O_NSZ)    /* [kind][dtype] : 12 */
#define O_BARWI (O_FLOP + O_NKIND * 2)
#define O_BARWG (O_BARWI + 1)
#define O_WG (O_BARWI + 2)
#define O_WI (O_BARWI + 3)
#define O_NLBIN 7
#define O_LDSB (O_BARWI + 4)          /* [dir][size][bank bin] : 42 */
#define O_FOOT (O_LDSB + 2 * O_NSZ * O_NLBIN) /* per array: |F|, |Fill| : 16 */
#define O_NOUT (O_FOOT + 2 * O_MAXARR)

enum { K_ADD, K_MUL, K_DIV, K_EXP, K_SPEC, K_FMA };
enum { D_LD, D_ST };

static const char *cls_name[O_NCLS] = {
    "0", "1", "1/2", "2/2", "1/3", "2/3", "3/3", "1/4", "2/4", "3/4", "4/4",
    "1/>4", "2/>4", "3/>4", "4/>4"};
static const char *kind_name[O_NKIND] = {"add", "mul", "div", "exp", "spec",
                                         "fma"};

typedef struct {
    int used, arr, dir, elem, vec;
    int64_t delta; /* flat element index change for local id 0 + 1 */
    int64_t count;
} site_t;

typedef struct {
    int64_t cells;
    uint8_t *touched;
    int64_t *diff; /* +1/-1 at run starts/ends of the gap-filling runs */
    int64_t difflen;
} arr_t;

typedef struct {
    site_t site[O_MAXSITE];
    arr_t arr[O_MAXARR];
    int narr;
    int64_t lds[2][O_NSZ];
    int64_t ldsb[2][O_NSZ][O_NLBIN];
    int64_t flop[O_NKIND][2];
    int64_t bar_wi, bar_wg, wg, wi;
    int err;
    char msg[200];
} sim_t;

/* parameters in this oracle's own order (see oracle/count.py) */
typedef struct {
    int64_t family, ebytes, op, n, m, l, wgx, wgy, T, s, gs, vec, reps, K, W,
        groups;
} oparams;

static void fail(sim_t *S, const char *m) {
    if (!S->err) {
        S->err = 1;
        snprintf(S->msg, sizeof S->msg, "%s", m);
    }
}

static int size_index(int bytes) {
    return bytes == 4 ? 0 : bytes == 8 ? 1 : bytes == 16 ? 2 : -1;
}

/* The gap-filling difference array is allocated when the array's first
 * access of stride >= 2 arrives (most arrays never need one): memory only,
 * the counts do not depend on it. */
static void new_array(sim_t *S, int a, int64_t cells) {
    S->arr[a].cells = cells;
    S->arr[a].touched = (uint8_t *)calloc((size_t)(cells > 0 ? cells : 1), 1);
    S->arr[a].difflen = 0;
    S->arr[a].diff = NULL;
    if (a + 1 > S->narr) S->narr = a + 1;
}

static void grow_diff(arr_t *A, int64_t need) {
    if (need < A->difflen) return;
    int64_t nl = A->diff ? A->difflen + A->difflen / 8 + 1024 : A->cells + 1024;
    if (nl <= need) nl = need + 1024;
    A->diff = (int64_t *)realloc(A->diff, (size_t)nl * 8);
    memset(A->diff + A->difflen, 0, (size_t)(nl - A->difflen) * 8);
    A->difflen = nl;
}

/* One global access event at site `site`: `idx` is the flat element index
 * of its first element, `idx_next` the same index expression evaluated
 * with local id 0 one larger. */
static void gacc(sim_t *S, int site, int a, int dir, int elem, int vec,
                 int64_t idx, int64_t idx_next) {
    site_t *t = &S->site[site];
    int64_t d = idx_next - idx;
    if (!t->used) {
        t->used = 1;
        t->arr = a;
        t->dir = dir;
        t->elem = elem;
        t->vec = vec;
        t->delta = d;
    } else if (t->delta != d || t->arr != a || t->dir != dir) {
        fail(S, "access site changes stride or array");
        return;
    }
    t->count++;
    arr_t *A = &S->arr[a];
    if (idx < 0 || idx + vec > A->cells) {
        fail(S, "access out of bounds");
        return;
    }
    for (int c = 0; c < vec; c++) A->touched[idx + c] = 1;
    int64_t ad = d < 0 ? -d : d;
    if (ad % vec) {
        fail(S, "lane stride is not a whole number of accesses");
        return;
    }
    int64_t s = ad / vec;
    if (s >= 2) {
        /* cells idx..idx+vec-1 each open a run of s*vec cells */
        int64_t end = idx + vec - 1 + s * vec;
        grow_diff(A, end + 1);
        A->diff[idx] += 1;
        A->diff[end] -= 1;
    }
}

/* `times` LDS accesses of `bytes` bytes at one site whose element index is
 * i0 for this work-item and i1 for the one with local id 0 one higher. */
static void lds(sim_t *S, int dir, int bytes, int64_t i0, int64_t i1, int64_t times) {
    int z = size_index(bytes);
    S->lds[dir][z] += times;
    int64_t words = (i1 - i0) * bytes / 4;
    if (words < 0) words = -words;
    int bin = 0;
    if (words) {
        int twos = 0;
        while (words % 2 == 0) {
            words /= 2;
            twos++;
        }
        bin = 1 + (twos < 5 ? twos : 5);
    }
    S->ldsb[dir][z][bin] += times;
}
static void flop(sim_t *S, int kind, int ebytes, int64_t times) {
    S->flop[kind][ebytes == 4 ? 0 : 1] += times;
}
/* a barrier reached by one work-item; lane0 says it is the group's first */
static void bar(sim_t *S, int lane0) {
    S->bar_wi++;
    if (lane0) S->bar_wg++;
}

/* ---------------------------------------------------------------- stream */
enum { ST_LOAD, ST_STORE, ST_COPY, ST_ADD4, ST_FILLED, ST_AXPBY };

static void sim_stream(sim_t *S, const oparams *p) {
    int64_t N = p->n, wg = p->wgx, s = p->s, gs = p->gs, vec = p->vec,
            U = p->reps;
    int e = (int)p->ebytes;
    if (wg <= 0 || N % wg) { fail(S, "n must be a multiple of wg"); return; }
    int64_t G = N / wg;
    if (p->op == ST_FILLED) {
        /* of every s cells the first c are read and summed left to right,
         * then added to the work-item's running sum */
        int64_t c = p->K;
        if (s < 2 || c < 1 || c > s || c >= O_MAXSITE) {
            fail(S, "filled needs 1 <= c <= s, s >= 2");
            return;
        }
        new_array(S, 0, s * G * wg * U);
        new_array(S, 1, N);
        for (int64_t g = 0; g < G; g++)
            for (int64_t l = 0; l < wg; l++) {
                for (int64_t u = 0; u < U; u++) {
                    int64_t j = (g * wg + l) + u * G * wg;
                    int64_t jn = (g * wg + l + 1) + u * G * wg;
                    for (int64_t q = 0; q < c; q++)
                        gacc(S, (int)q, 0, D_LD, e, 1, s * j + q, s * jn + q);
                    flop(S, K_ADD, e, c - 1); /* x0 + x1 + ... + x_{c-1} */
                    flop(S, K_ADD, e, 1);     /* acc += */
                }
                gacc(S, O_MAXSITE - 1, 1, D_ST, e, 1, g * wg + l, g * wg + l + 1);
            }
    } else {
        int64_t span = G * gs * wg * s * U * vec;
        int na = p->op == ST_ADD4 ? 5 : p->op == ST_AXPBY ? 3 : p->op == ST_COPY ? 2 : 1;
        for (int a = 0; a < na; a++) new_array(S, a, span);
        for (int64_t g = 0; g < G; g++)
            for (int64_t l = 0; l < wg; l++)
                for (int64_t u = 0; u < U; u++) {
                    int64_t x = vec * (((g * gs) * wg + l) * s + u * G * gs * wg * s);
                    int64_t xn = vec * (((g * gs) * wg + l + 1) * s + u * G * gs * wg * s);
                    switch (p->op) {
                    case ST_LOAD: /* summed in a register, never stored */
                        gacc(S, 0, 0, D_LD, e, (int)vec, x, xn);
                        flop(S, K_ADD, e, vec);
                        break;
                    case ST_STORE:
                        gacc(S, 0, 0, D_ST, e, (int)vec, x, xn);
                        break;
                    case ST_COPY:
                        gacc(S, 0, 0, D_LD, e, (int)vec, x, xn);
                        gacc(S, 1, 1, D_ST, e, (int)vec, x, xn);
                        break;
                    case ST_ADD4:
                        for (int a = 0; a < 4; a++)
                            gacc(S, a, a, D_LD, e, (int)vec, x, xn);
                        gacc(S, 4, 4, D_ST, e, (int)vec, x, xn);
                        flop(S, K_ADD, e, 3 * vec);
                        break;
                    case ST_AXPBY: /* out = alpha x + beta y */
                        gacc(S, 0, 0, D_LD, e, (int)vec, x, xn);
                        gacc(S, 1, 1, D_LD, e, (int)vec, x, xn);
                        gacc(S, 2, 2, D_ST, e, (int)vec, x, xn);
                        flop(S, K_MUL, e, 2 * vec);
                        flop(S, K_ADD, e, vec);
                        break;
                    default:
                        fail(S, "bad stream op");
                        return;
                    }
                }
    }
    S->wg += G;
    S->wi += G * wg;
}

/* ------------------------------------------------------------------- lds */
static void sim_lds(sim_t *S, const oparams *p) {
    int64_t G = p->groups, wg = p->wgx, R = p->reps, W = p->W;
    if (W % wg) { fail(S, "W must be a multiple of wg"); return; }
    new_array(S, 0, G * wg);
    for (int64_t g = 0; g < G; g++)
        for (int64_t l = 0; l < wg; l++) {
            int64_t b = p->s; /* bank stride: lds[(l*b + r) mod W] */
            if (p->op == 0) { /* read */
                for (int64_t c = 0; c < W / wg; c++)
                    lds(S, D_ST, 4, c * wg + l, c * wg + l + 1, 1);
                bar(S, l == 0);
                lds(S, D_LD, 4, l * b, (l + 1) * b, R);
                flop(S, K_ADD, 4, R);
            } else { /* write */
                lds(S, D_ST, 4, l * b, (l + 1) * b, R);
                bar(S, l == 0);
                lds(S, D_LD, 4, l * b, (l + 1) * b, 1);
            }
            gacc(S, 0, 0, D_ST, 4, 1, g * wg + l, g * wg + l + 1);
        }
    S->wg += G;
    S->wi += G * wg;
}

/* --------------------------------------------------------- fma and rsqrt */
/* mode 0: FMA chain; 1: rsqrt chain y = rsqrt(y*y + d); 2: division
 * chain y = d / (y*y + 1); 3: exponential chain y = exp(-(y*y)) */
static void sim_fma(sim_t *S, const oparams *p, int rsqrt) {
    int64_t N = p->n, wg = p->wgx, F = p->reps, K = p->K;
    int e = (int)p->ebytes;
    if (N % wg || K <= 0 || F % K) { fail(S, "bad fma shape"); return; }
    new_array(S, 0, N);
    new_array(S, 1, N);
    for (int64_t i = 0; i < N; i++) {
        gacc(S, 0, 0, D_LD, e, 1, i, i + 1);
        for (int64_t f = 0; f < F; f++) {
            if (rsqrt == 1) { /* y = rsqrt(y*y + d) */
                flop(S, K_MUL, e, 1);
                flop(S, K_ADD, e, 1);
                flop(S, K_SPEC, e, 1);
            } else if (rsqrt == 2) { /* y = d / (y*y + 1) */
                flop(S, K_MUL, e, 1);
                flop(S, K_ADD, e, 1);
                flop(S, K_DIV, e, 1);
            } else if (rsqrt == 3) { /* y = exp(-(y*y)): negation not counted */
                flop(S, K_MUL, e, 1);
                flop(S, K_EXP, e, 1);
            } else {
                flop(S, K_FMA, e, 1);
            }
        }
        flop(S, K_ADD, e, K - 1); /* chains summed */
        gacc(S, 1, 1, D_ST, e, 1, i, i + 1);
    }
    S->wg += N / wg;
    S->wi += N;
}

/* ------------------------------------------------------ barrier / empty */
static void sim_barrier(sim_t *S, const oparams *p) {
    int64_t G = p->groups, wg = p->wgx, B = p->reps;
    new_array(S, 0, G * wg);
    for (int64_t g = 0; g < G; g++)
        for (int64_t l = 0; l < wg; l++) {
            for (int64_t b = 0; b < B; b++) bar(S, l == 0);
            gacc(S, 0, 0, D_ST, 4, 1, g * wg + l, g * wg + l + 1);
        }
    S->wg += G;
    S->wi += G * wg;
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static void sim_empty(sim_t *S, const oparams *p) {
    int64_t gx = cdiv(p->n, p->wgx), gy = cdiv(p->n, p->wgy);
    S->wg += gx * gy;
    S->wi += gx * gy * p->wgx * p->wgy;
}

/* ---------------------------------------------------------------- matmul */
static void sim_matmul(sim_t *S, const oparams *p) {
    int64_t n = p->n, m = p->m, L = p->l, T = p->T;
    int64_t GX = cdiv(L, T), GY = cdiv(n, T), KT = cdiv(m, T);
    new_array(S, 0, n * m);
    new_array(S, 1, m * L);
    new_array(S, 2, n * L);
    for (int64_t gy = 0; gy < GY; gy++)
        for (int64_t gx = 0; gx < GX; gx++)
            for (int64_t ly = 0; ly < T; ly++)
                for (int64_t lx = 0; lx < T; lx++) {
                    int64_t row = gy * T + ly, col = gx * T + lx;
                    int lane0 = lx == 0 && ly == 0;
                    if (p->op == 0) { /* tiled, LDS prefetch */
                        for (int64_t kt = 0; kt < KT; kt++) {
                            if (row < n && kt * T + lx < m)
                                gacc(S, 0, 0, D_LD, 4, 1, row * m + kt * T + lx,
                                     row * m + kt * T + lx + 1);
                            lds(S, D_ST, 4, ly * T + lx, ly * T + lx + 1, 1); /* As[ly][lx] */
                            if (kt * T + ly < m && col < L)
                                gacc(S, 1, 1, D_LD, 4, 1, (kt * T + ly) * L + col,
                                     (kt * T + ly) * L + col + 1);
                            /* Bs[ly][lx], rows of T + 1 */
                            lds(S, D_ST, 4, ly * (T + 1) + lx, ly * (T + 1) + lx + 1, 1);
                            bar(S, lane0);
                            for (int64_t kk = 0; kk < T; kk++) {
                                lds(S, D_LD, 4, ly * T + kk, ly * T + kk, 1); /* As[ly][kk] */
                                lds(S, D_LD, 4, kk * (T + 1) + lx, kk * (T + 1) + lx + 1, 1);
                                flop(S, K_FMA, 4, 1);
                            }
                            bar(S, lane0);
                        }
                        if (row < n && col < L)
                            gacc(S, 2, 2, D_ST, 4, 1, row * L + col, row * L + col + 1);
                    } else { /* naive: one inner product per work-item */
                        if (row < n && col < L) {
                            for (int64_t k = 0; k < m; k++) {
                                gacc(S, 0, 0, D_LD, 4, 1, row * m + k, row * m + k);
                                gacc(S, 1, 1, D_LD, 4, 1, k * L + col, k * L + col + 1);
                                flop(S, K_FMA, 4, 1);
                            }
                            gacc(S, 2, 2, D_ST, 4, 1, row * L + col, row * L + col + 1);
                        }
                    }
                }
    S->wg += GX * GY;
    S->wi += GX * GY * T * T;
}

/* ------------------------------------------------------------- transpose */
static void sim_transpose(sim_t *S, const oparams *p) {
    int64_t n = p->n, T = p->T, G = cdiv(n, T);
    new_array(S, 0, n * n);
    new_array(S, 1, n * n);
    for (int64_t gy = 0; gy < G; gy++)
        for (int64_t gx = 0; gx < G; gx++)
            for (int64_t ly = 0; ly < T; ly++)
                for (int64_t lx = 0; lx < T; lx++) {
                    int64_t r = gy * T + ly, c = gx * T + lx;
                    if (p->op == 0) { /* tiled through LDS */
                        if (r < n && c < n) {
                            gacc(S, 0, 0, D_LD, 4, 1, r * n + c, r * n + c + 1);
                            /* tile[ly][lx], rows of T + 1 */
                            lds(S, D_ST, 4, ly * (T + 1) + lx, ly * (T + 1) + lx + 1, 1);
                        }
                        bar(S, lx == 0 && ly == 0);
                        int64_t r2 = gx * T + ly, c2 = gy * T + lx;
                        if (r2 < n && c2 < n) {
                            lds(S, D_LD, 4, lx * (T + 1) + ly, (lx + 1) * (T + 1) + ly, 1);
                            gacc(S, 1, 1, D_ST, 4, 1, r2 * n + c2, r2 * n + c2 + 1);
                        }
                    } else if (r < n && c < n) {
                        if (p->op == 1) { /* writes coalesced, reads strided */
                            gacc(S, 0, 0, D_LD, 4, 1, c * n + r, (c + 1) * n + r);
                            gacc(S, 1, 1, D_ST, 4, 1, r * n + c, r * n + c + 1);
                        } else { /* reads coalesced, writes strided */
                            gacc(S, 0, 0, D_LD, 4, 1, r * n + c, r * n + c + 1);
                            gacc(S, 1, 1, D_ST, 4, 1, c * n + r, (c + 1) * n + r);
                        }
                    }
                }
    S->wg += G * G;
    S->wi += G * G * T * T;
}

/* --------------------------------------------------------------- stencil */
static void sim_stencil(sim_t *S, const oparams *p) {
    int64_t n = p->n, T = p->T, G = cdiv(n, T), P = n + 2;
    int64_t Q = T + 2; /* the LDS tile: rows of T + 2 with the halo */
    int e = (int)p->ebytes;
    new_array(S, 0, P * P);
    new_array(S, 1, n * n);
    for (int64_t gy = 0; gy < G; gy++)
        for (int64_t gx = 0; gx < G; gx++)
            for (int64_t ly = 0; ly < T; ly++)
                for (int64_t lx = 0; lx < T; lx++) {
                    int64_t i = gy * T + ly, j = gx * T + lx;
                    int in = i < n && j < n;
                    /* the tile, then its four halo edges */
                    if (in) {
                        gacc(S, 0, 0, D_LD, e, 1, (i + 1) * P + j + 1, (i + 1) * P + j + 2);
                        lds(S, D_ST, e, (ly + 1) * Q + lx + 1, (ly + 1) * Q + lx + 2, 1);
                    }
                    if (ly == 0 && j < n) {
                        gacc(S, 1, 0, D_LD, e, 1, i * P + j + 1, i * P + j + 2);
                        lds(S, D_ST, e, lx + 1, lx + 2, 1);
                    }
                    if (ly == T - 1 && in) {
                        gacc(S, 2, 0, D_LD, e, 1, (i + 2) * P + j + 1, (i + 2) * P + j + 2);
                        lds(S, D_ST, e, (T + 1) * Q + lx + 1, (T + 1) * Q + lx + 2, 1);
                    }
                    if (ly < T - 1 && i == n - 1 && j < n) {
                        gacc(S, 3, 0, D_LD, e, 1, (i + 2) * P + j + 1, (i + 2) * P + j + 2);
                        lds(S, D_ST, e, (ly + 2) * Q + lx + 1, (ly + 2) * Q + lx + 2, 1);
                    }
                    if (lx == 0 && i < n) {
                        gacc(S, 4, 0, D_LD, e, 1, (i + 1) * P + j, (i + 1) * P + j + 1);
                        lds(S, D_ST, e, (ly + 1) * Q, (ly + 1) * Q, 1); /* column 0 */
                    }
                    if (lx == T - 1 && in) {
                        gacc(S, 5, 0, D_LD, e, 1, (i + 1) * P + j + 2, (i + 1) * P + j + 3);
                        lds(S, D_ST, e, (ly + 1) * Q + T + 1, (ly + 1) * Q + T + 1, 1);
                    }
                    if (lx < T - 1 && j == n - 1 && i < n) {
                        gacc(S, 6, 0, D_LD, e, 1, (i + 1) * P + j + 2, (i + 1) * P + j + 3);
                        lds(S, D_ST, e, (ly + 1) * Q + lx + 2, (ly + 1) * Q + lx + 3, 1);
                    }
                    bar(S, lx == 0 && ly == 0);
                    if (in) {
                        /* the point, north, south, west, east */
                        lds(S, D_LD, e, (ly + 1) * Q + lx + 1, (ly + 1) * Q + lx + 2, 1);
                        lds(S, D_LD, e, ly * Q + lx + 1, ly * Q + lx + 2, 1);
                        lds(S, D_LD, e, (ly + 2) * Q + lx + 1, (ly + 2) * Q + lx + 2, 1);
                        lds(S, D_LD, e, (ly + 1) * Q + lx, (ly + 1) * Q + lx + 1, 1);
                        lds(S, D_LD, e, (ly + 1) * Q + lx + 2, (ly + 1) * Q + lx + 3, 1);
                        flop(S, K_ADD, e, 4); /* N+S, +W, +E, + h^2 c^2 */
                        flop(S, K_MUL, e, 3); /* c*c, h^2*(.), 0.25*(.) */
                        gacc(S, 7, 1, D_ST, e, 1, i * n + j, i * n + j + 1);
                    }
                }
    S->wg += G * G;
    S->wi += G * G * T * T;
}

/* ----------------------------------------------------------------- nbody */
static void sim_nbody(sim_t *S, const oparams *p) {
    int64_t N = p->n, Gs = p->wgx, G = cdiv(N, Gs);
    new_array(S, 0, 3 * N);
    new_array(S, 1, N);
    for (int64_t g = 0; g < G; g++)
        for (int64_t l = 0; l < Gs; l++) {
            int64_t i = g * Gs + l;
            if (i < N)
                for (int c = 0; c < 3; c++)
                    gacc(S, c, 0, D_LD, 4, 1, 3 * i + c, 3 * (i + 1) + c);
            for (int64_t jb = 0; jb < G; jb++) {
                int64_t j = jb * Gs + l;
                if (j < N)
                    for (int c = 0; c < 3; c++) {
                        gacc(S, 3 + c, 0, D_LD, 4, 1, 3 * j + c, 3 * (j + 1) + c);
                        lds(S, D_ST, 4, c * Gs + l, c * Gs + l + 1, 1); /* sh[c*G + l] */
                    }
                bar(S, l == 0);
                for (int64_t jj = 0; jj < Gs; jj++)
                    if (jb * Gs + jj < N) {
                        for (int c = 0; c < 3; c++) /* sh[c*G + jj], one word for all */
                            lds(S, D_LD, 4, c * Gs + jj, c * Gs + jj, 1);
                        flop(S, K_ADD, 4, 6); /* 3 sub, 2 add in r^2, 1 into the block's partial */
                        flop(S, K_MUL, 4, 3);
                        flop(S, K_SPEC, 4, 1); /* rsqrt, self pair masked by select */
                    }
                flop(S, K_ADD, 4, 1); /* the block's partial added to the total */
                bar(S, l == 0);
            }
            if (i < N) gacc(S, 6, 1, D_ST, 4, 1, i, i + 1);
        }
    S->wg += G;
    S->wi += G * Gs;
}

/* ----------------------------------------------------------------- conv */
/* Three 7x7 filters over three RGB images (Sec. 5): r[i][j][x][y] = sum over
 * u, v in [0,7), c < 3 of img[i][x+6-u][y+6-v][c] * filt[j][u][v][c];
 * images (n+6)^2 x 3 (channel fastest), T x T work-groups, one per output
 * tile and (image, filter) pair; the (T+6)^2 x 3 image tile and the filter
 * are staged through LDS. */
static void sim_conv(sim_t *S, const oparams *p) {
    int64_t n = p->n, T = p->T, P = n + 6, G = cdiv(n, T), TT = T + 6;
    int64_t KF = cdiv(147, T * T), KA = cdiv(TT, T);
    new_array(S, 0, 3 * P * P * 3);
    new_array(S, 1, 3 * 147);
    new_array(S, 2, 9 * n * n);
    for (int64_t zi = 0; zi < 3; zi++)
        for (int64_t zj = 0; zj < 3; zj++)
            for (int64_t gy = 0; gy < G; gy++)
                for (int64_t gx = 0; gx < G; gx++)
                    for (int64_t ly = 0; ly < T; ly++)
                        for (int64_t lx = 0; lx < T; lx++) {
                            int lane0 = lx == 0 && ly == 0;
                            for (int64_t k = 0; k < KF; k++) {
                                int64_t t = k * T * T + ly * T + lx;
                                if (t < 147) {
                                    gacc(S, 0, 1, D_LD, 4, 1, zj * 147 + t, zj * 147 + t + 1);
                                    lds(S, D_ST, 4, t, t + 1, 1); /* fl[t] */
                                }
                            }
                            for (int64_t a = 0; a < KA; a++)
                                for (int64_t b = 0; b < KA; b++) {
                                    int64_t r = a * T + ly, q = b * T + lx;
                                    int64_t X = gy * T + r, Y = gx * T + q;
                                    if (r < TT && q < TT && X < P && Y < P)
                                        for (int64_t c = 0; c < 3; c++) {
                                            int64_t id = ((zi * P + X) * P + Y) * 3 + c;
                                            gacc(S, 1 + (int)c, 0, D_LD, 4, 1, id, id + 3);
                                            /* tile[r][q][c], channel fastest */
                                            lds(S, D_ST, 4, (r * TT + q) * 3 + c,
                                                (r * TT + q + 1) * 3 + c, 1);
                                        }
                                }
                            bar(S, lane0);
                            int64_t x = gy * T + ly, y = gx * T + lx;
                            if (x < n && y < n) {
                                for (int64_t u = 0; u < 7; u++)
                                    for (int64_t v = 0; v < 7; v++) {
                                        for (int64_t c = 0; c < 3; c++) {
                                            int64_t a0 = ((ly + 6 - u) * TT + lx + 6 - v) * 3 + c;
                                            lds(S, D_LD, 4, a0, a0 + 3, 1); /* tile */
                                            int64_t f0 = (u * 7 + v) * 3 + c;
                                            lds(S, D_LD, 4, f0, f0, 1);     /* fl */
                                        }
                                        flop(S, K_FMA, 4, 3);
                                    }
                                int64_t o = ((zi * 3 + zj) * n + x) * n + y;
                                gacc(S, 4, 2, D_ST, 4, 1, o, o + 1);
                            }
                        }
    S->wg += 9 * G * G;
    S->wi += 9 * G * G * T * T;
}

/* ------------------------------------------------------ classification */
static int class_index(int64_t s, int64_t F, int64_t Fill) {
    if (s == 0) return 0;
    if (s == 1) return 1;
    int64_t q = s < 4 ? s : 4;
    int64_t k = (q * F + Fill - 1) / Fill; /* ceil(q F / Fill) */
    if (k < 1) k = 1;
    if (k > q) k = q;
    int base = s == 2 ? 2 : s == 3 ? 4 : s == 4 ? 7 : 11;
    return base + (int)(k - 1);
}

static void finish(sim_t *S, int64_t *out) {
    memset(out, 0, sizeof(int64_t) * O_NOUT);
    int64_t Fc[O_MAXARR] = {0}, Fill[O_MAXARR] = {0};
    for (int a = 0; a < S->narr; a++) {
        arr_t *A = &S->arr[a];
        int64_t run = 0, f = 0, fill = 0;
        int64_t len = A->difflen > A->cells ? A->difflen : A->cells;
        for (int64_t x = 0; x < len; x++) {
            if (x < A->difflen) run += A->diff[x];
            int t = x < A->cells ? A->touched[x] : 0;
            f += t;
            fill += (t || run > 0);
        }
        Fc[a] = f;
        Fill[a] = fill;
        out[O_FOOT + 2 * a] = f;
        out[O_FOOT + 2 * a + 1] = fill;
    }
    for (int j = 0; j < O_MAXSITE; j++) {
        site_t *t = &S->site[j];
        if (!t->used) continue;
        int64_t ad = t->delta < 0 ? -t->delta : t->delta;
        int64_t s = ad / t->vec;
        int si = size_index(t->elem * t->vec);
        if (si < 0) { fail(S, "unsupported access size"); return; }
        int c = class_index(s, Fc[t->arr], Fill[t->arr] ? Fill[t->arr] : 1);
        out[O_GACC + (t->dir * O_NSZ + si) * O_NCLS + c] += t->count;
    }
    for (int d = 0; d < 2; d++)
        for (int z = 0; z < O_NSZ; z++) {
            out[O_LDS + d * O_NSZ + z] = S->lds[d][z];
            for (int b = 0; b < O_NLBIN; b++)
                out[O_LDSB + (d * O_NSZ + z) * O_NLBIN + b] = S->ldsb[d][z][b];
        }
    for (int k = 0; k < O_NKIND; k++)
        for (int d = 0; d < 2; d++) out[O_FLOP + k * 2 + d] = S->flop[k][d];
    out[O_BARWI] = S->bar_wi;
    out[O_BARWG] = S->bar_wg;
    out[O_WG] = S->wg;
    out[O_WI] = S->wi;
}

/* ------------------------------------------------------------ C entries */
int oracle_nout(void) { return O_NOUT; }

/* Name of output slot i, e.g. "gld.4.1/2", "lst.8", "fma.f32", "bar.wi",
 * "foot.F.0" (|F| of array 0), "foot.fill.0". */
int oracle_name(int i, char *buf, int cap) {
    static const char *szn[O_NSZ] = {"4", "8", "16"};
    if (i < 0 || i >= O_NOUT) return -1;
    if (i < O_LDS) {
        int d = i / (O_NSZ * O_NCLS), r = i % (O_NSZ * O_NCLS);
        snprintf(buf, cap, "%s.%s.%s", d ? "gst" : "gld", szn[r / O_NCLS],
                 cls_name[r % O_NCLS]);
    } else if (i < O_FLOP) {
        int r = i - O_LDS;
        snprintf(buf, cap, "%s.%s", r / O_NSZ ? "lst" : "lld", szn[r % O_NSZ]);
    } else if (i < O_BARWI) {
        int r = i - O_FLOP;
        snprintf(buf, cap, "%s.%s", kind_name[r / 2], r % 2 ? "f64" : "f32");
    } else if (i == O_BARWI) {
        snprintf(buf, cap, "bar.wi");
    } else if (i == O_BARWG) {
        snprintf(buf, cap, "bar.wg");
    } else if (i == O_WG) {
        snprintf(buf, cap, "wg");
    } else if (i == O_WI) {
        snprintf(buf, cap, "wi");
    } else if (i < O_FOOT) {
        static const char *bn[O_NLBIN] = {"b0", "b1", "b2", "b4", "b8", "b16", "b32"};
        int r = i - O_LDSB, dz = r / O_NLBIN;
        snprintf(buf, cap, "%s.%s.%s", dz / O_NSZ ? "lst" : "lld", szn[dz % O_NSZ], bn[r % O_NLBIN]);
    } else {
        int r = i - O_FOOT;
        snprintf(buf, cap, "foot.%s.%d", r % 2 ? "fill" : "F", r / 2);
    }
    return 0;
}

/* Count one variant.  p: 16 int64 parameters in oparams order.  Returns 0
 * on success, -1 on error (message in msg). */
int oracle_count(const int64_t *p_in, int64_t *out, char *msg, int msgcap) {
    oparams p;
    memcpy(&p, p_in, sizeof p);
    sim_t *S = (sim_t *)calloc(1, sizeof(sim_t));
    switch (p.family) {
    case 0: sim_stream(S, &p); break;
    case 1: sim_lds(S, &p); break;
    case 2: sim_fma(S, &p, 0); break;
    case 3: sim_fma(S, &p, 1); break;
    case 4: sim_barrier(S, &p); break;
    case 5: sim_empty(S, &p); break;
    case 6: sim_matmul(S, &p); break;
    case 7: sim_transpose(S, &p); break;
    case 8: sim_stencil(S, &p); break;
    case 9: sim_nbody(S, &p); break;
    case 10: sim_fma(S, &p, p.op == 0 ? 2 : 3); break;
    case 11: sim_conv(S, &p); break;
    default: fail(S, "unknown family");
    }
    if (!S->err) finish(S, out);
    int rc = S->err ? -1 : 0;
    if (msg && msgcap > 0) snprintf(msg, msgcap, "%s", S->err ? S->msg : "");
    for (int a = 0; a < S->narr; a++) {
        free(S->arr[a].touched);
        free(S->arr[a].diff);
    }
    free(S);
    return rc;
}

/* Textbook stride cases: one array of `cells` cells, sites given as
 * flat index = coef * i + off over i in [0, n), each of `vec` elements of
 * `elem` bytes.  Writes the class index of each site to cls[]. */
int oracle_classify_1d(int64_t cells, int64_t n, int nsite, const int64_t *coef,
                       const int64_t *off, int elem, int vec, int *cls) {
    sim_t *S = (sim_t *)calloc(1, sizeof(sim_t));
    new_array(S, 0, cells);
    for (int64_t i = 0; i < n; i++)
        for (int j = 0; j < nsite && j < O_MAXSITE; j++)
            gacc(S, j, 0, D_LD, elem, vec, coef[j] * i + off[j],
                 coef[j] * (i + 1) + off[j]);
    int rc = 0;
    if (!S->err) {
        int64_t out[O_NOUT];
        finish(S, out);
        for (int j = 0; j < nsite; j++) {
            site_t *t = &S->site[j];
            int64_t ad = t->delta < 0 ? -t->delta : t->delta;
            cls[j] = class_index(ad / vec, out[O_FOOT], out[O_FOOT + 1]);
        }
    } else {
        rc = -1;
    }
    free(S->arr[0].touched);
    free(S->arr[0].diff);
    free(S);
    return rc;
}

/* ----------------------------------------------- FMA-chain output oracle */
/* chain k: c = a, then F/K times c = fma(c, a, (k+1)/64); out = sum of
 * chains left to right.  fmaf/fma of the C library round once (IEEE). */
#include <math.h>
void oracle_fma_chain_f32(const float *in, float *out, int64_t n, int64_t F,
                          int64_t K) {
    for (int64_t i = 0; i < n; i++) {
        float a = in[i], c[64];
        for (int64_t k = 0; k < K; k++) c[k] = a;
        for (int64_t f = 0; f < F / K; f++)
            for (int64_t k = 0; k < K; k++)
                c[k] = fmaf(c[k], a, (float)(k + 1) * 0.015625f);
        float s = c[0];
        for (int64_t k = 1; k < K; k++) s = s + c[k];
        out[i] = s;
    }
}

void oracle_fma_chain_f64(const double *in, double *out, int64_t n, int64_t F,
                          int64_t K) {
    for (int64_t i = 0; i < n; i++) {
        double a = in[i], c[64];
        for (int64_t k = 0; k < K; k++) c[k] = a;
        for (int64_t f = 0; f < F / K; f++)
            for (int64_t k = 0; k < K; k++)
                c[k] = fma(c[k], a, (double)(k + 1) * 0.015625);
        double s = c[0];
        for (int64_t k = 1; k < K; k++) s = s + c[k];
        out[i] = s;
    }
}
