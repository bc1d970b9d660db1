// The kernel suite: performance-instructive kernels (Sec. 4.1) and the
// test kernels whose run times the model predicts (Sec. 5), hand-written
// for gfx950.  Every kernel's structure is mirrored statement by statement
// by its descriptor in desc.h.
//
// Built with -ffp-contract=off: products and sums stay separate roundings
// (the FMA-based kernels call fmaf/fma explicitly), so outputs follow the
// stated operation order exactly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm.h"
#include "suite.h"

namespace pm {

template <typename T, int V> struct Vec;
template <> struct Vec<float, 1> { using t = float; };
template <> struct Vec<float, 2> { using t = float2; };
template <> struct Vec<float, 4> { using t = float4; };
template <> struct Vec<double, 1> { using t = double; };
template <> struct Vec<double, 2> { using t = double2; };

template <typename T> __device__ inline T comp(T v, int) { return v; }
__device__ inline float comp(float2 v, int c) { return c ? v.y : v.x; }
__device__ inline float comp(float4 v, int c) { return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w; }
__device__ inline double comp(double2 v, int c) { return c ? v.y : v.x; }

// Streaming accesses: the non-temporal cache hint on a load or store whose
// line no later access of the kernel touches.
template <typename T> __device__ inline T ld_nt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ inline void st_nt(T v, T *p) { __builtin_nontemporal_store(v, p); }
typedef float nf2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef double nd2 __attribute__((ext_vector_type(2)));
template <> __device__ inline float2 ld_nt(const float2 *p) {
    const nf2 r = __builtin_nontemporal_load((const nf2 *)p);
    return make_float2(r[0], r[1]);
}
template <> __device__ inline float4 ld_nt(const float4 *p) {
    const nf4 r = __builtin_nontemporal_load((const nf4 *)p);
    return make_float4(r[0], r[1], r[2], r[3]);
}
template <> __device__ inline double2 ld_nt(const double2 *p) {
    const nd2 r = __builtin_nontemporal_load((const nd2 *)p);
    return make_double2(r[0], r[1]);
}
template <> __device__ inline void st_nt(float2 v, float2 *p) {
    __builtin_nontemporal_store(nf2{v.x, v.y}, (nf2 *)p);
}
template <> __device__ inline void st_nt(float4 v, float4 *p) {
    __builtin_nontemporal_store(nf4{v.x, v.y, v.z, v.w}, (nf4 *)p);
}
template <> __device__ inline void st_nt(double2 v, double2 *p) {
    __builtin_nontemporal_store(nd2{v.x, v.y}, (nd2 *)p);
}
// A plain or (NT) streaming access.
template <bool NT, typename T> __device__ inline T ld(const T *p) { return NT ? ld_nt(p) : *p; }
template <bool NT, typename T> __device__ inline void st(T v, T *p) {
    if (NT) st_nt(v, p);
    else *p = v;
}

template <typename VT, typename T> __device__ inline VT vset(T *a);
template <> __device__ inline float vset<float, float>(float *a) { return a[0]; }
template <> __device__ inline float2 vset<float2, float>(float *a) { return make_float2(a[0], a[1]); }
template <> __device__ inline float4 vset<float4, float>(float *a) { return make_float4(a[0], a[1], a[2], a[3]); }
template <> __device__ inline double vset<double, double>(double *a) { return a[0]; }
template <> __device__ inline double2 vset<double2, double>(double *a) { return make_double2(a[0], a[1]); }

// ----------------------------------------------------------------- stream
// Access u of work-item (g, l) is element vector number
// ((g*gs)*wg + l)*s + u*G*gs*wg*s (units of VEC elements).  NT: every
// access carries the streaming hint (no element is touched twice).
template <typename T, int VEC, int OP, bool NT>
__global__ void k_stream(T *__restrict__ x0, T *__restrict__ x1, T *__restrict__ x2,
                         T *__restrict__ x3, T *__restrict__ x4, int64_t G, int64_t s,
                         int64_t gs, int U, T sentinel) {
    using VT = typename Vec<T, VEC>::t;
    const int64_t wg = blockDim.x, g = blockIdx.x, l = threadIdx.x;
    const int64_t base = ((g * gs) * wg + l) * s;
    const int64_t ust = G * gs * wg * s;
    T acc = 0;
#pragma unroll 4
    for (int u = 0; u < U; u++) {
        int64_t e = base + u * ust;
        if (OP == PM_STREAM_LOAD) {
            VT a = ld<NT>((const VT *)x0 + e);
#pragma unroll
            for (int c = 0; c < VEC; c++) acc += comp(a, c);
        } else if (OP == PM_STREAM_STORE) {
            T t[VEC];
#pragma unroll
            for (int c = 0; c < VEC; c++) t[c] = (T)(e * VEC + c);
            st<NT>(vset<VT, T>(t), (VT *)x0 + e);
        } else if (OP == PM_STREAM_COPY) {
            st<NT>(ld<NT>((const VT *)x0 + e), (VT *)x1 + e);
        } else if (OP == PM_STREAM_AXPBY) {
            VT a = ld<NT>((const VT *)x0 + e), b = ld<NT>((const VT *)x1 + e);
            T t[VEC];
#pragma unroll
            for (int q = 0; q < VEC; q++)
                t[q] = (T)0.75 * comp(a, q) + (T)(-1.25) * comp(b, q);
            st<NT>(vset<VT, T>(t), (VT *)x2 + e);
        } else {  // add4
            VT a = ld<NT>((const VT *)x0 + e), b = ld<NT>((const VT *)x1 + e);
            VT c = ld<NT>((const VT *)x2 + e), d = ld<NT>((const VT *)x3 + e);
            T t[VEC];
#pragma unroll
            for (int q = 0; q < VEC; q++)
                t[q] = (comp(a, q) + comp(b, q)) + (comp(c, q) + comp(d, q));
            st<NT>(vset<VT, T>(t), (VT *)x4 + e);
        }
    }
    // never true (sentinel is NaN): keeps the loads without storing
    if (OP == PM_STREAM_LOAD && acc == sentinel) x1[g * wg + l] = acc;
}

// filled: of every s consecutive cells the first c are read (lane stride
// s, c accesses per group of s cells) and summed left to right,
// ((x0 + x1) + x2) + ..., into a running sum.
template <typename T>
__global__ void k_filled(const T *__restrict__ x, T *__restrict__ out, int64_t G, int U,
                         int s, int c) {
    const int64_t wg = blockDim.x;
    const int64_t i = (int64_t)blockIdx.x * wg + threadIdx.x;
    T acc = 0;
    for (int u = 0; u < U; u++) {
        const T *p = x + (i + (int64_t)u * G * wg) * s;
        T t = p[0];
        for (int q = 1; q < c; q++) t = t + p[q];
        acc = acc + t;
    }
    out[i] = acc;
}

// -------------------------------------------------------------------- LDS
__global__ void k_lds_read(float *out, int b, int R, int W) {
    extern __shared__ float lds[];
    const int l = threadIdx.x, wg = blockDim.x;
    for (int c = 0; c < W / wg; c++) lds[c * wg + l] = (float)(c * wg + l);
    __syncthreads();
    float acc = 0.f;
    for (int r = 0; r < R; r++) acc += lds[(l * b + r) & (W - 1)];
    out[(int64_t)blockIdx.x * wg + l] = acc;
}

__global__ void k_lds_write(float *out, int b, int R, int W) {
    extern __shared__ float lds[];
    const int l = threadIdx.x, wg = blockDim.x;
    for (int r = 0; r < R; r++) {
        int a = (l * b + r) & (W - 1);
        lds[a] = (float)a;
    }
    __syncthreads();
    out[(int64_t)blockIdx.x * wg + l] = lds[(l * b) & (W - 1)];
}

// ------------------------------------------------------------- FMA chains
template <typename T> __device__ inline T fmaT(T a, T b, T c);
template <> __device__ inline float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ inline double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T, int K>
__global__ void k_fma(const T *in, T *out, int F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const T a = in[i];
    T c[K];
#pragma unroll
    for (int k = 0; k < K; k++) c[k] = a;
    for (int f = 0; f < F / K; f++) {
#pragma unroll
        for (int k = 0; k < K; k++) c[k] = fmaT(c[k], a, (T)(k + 1) * (T)0.015625);
    }
    T s = c[0];
#pragma unroll
    for (int k = 1; k < K; k++) s = s + c[k];
    out[i] = s;
}

template <int K>
__global__ void k_rsqrt(const float *in, float *out, int F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float a = in[i];
    float y[K];
#pragma unroll
    for (int k = 0; k < K; k++) y[k] = a;
    for (int f = 0; f < F / K; f++) {
#pragma unroll
        for (int k = 0; k < K; k++) y[k] = rsqrtf(y[k] * y[k] + (float)(k + 1));
    }
    float s = y[0];
#pragma unroll
    for (int k = 1; k < K; k++) s = s + y[k];
    out[i] = s;
}

// division chains y = (k+1) / (y*y + 1) and exponential chains y = exp(-(y*y))
template <typename T> __device__ inline T expT(T x);
template <> __device__ inline float expT(float x) { return expf(x); }
template <> __device__ inline double expT(double x) { return exp(x); }

template <typename T, int K, int OP>
__global__ void k_arith(const T *in, T *out, int F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const T a = in[i];
    T y[K];
#pragma unroll
    for (int k = 0; k < K; k++) y[k] = a;
    for (int f = 0; f < F / K; f++) {
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (OP == PM_ARITH_DIV) y[k] = (T)(k + 1) / (y[k] * y[k] + (T)1);
            else y[k] = expT(-(y[k] * y[k]));
        }
    }
    T s = y[0];
#pragma unroll
    for (int k = 1; k < K; k++) s = s + y[k];
    out[i] = s;
}

// --------------------------------------------------------- convolution
// r[i][j][x][y] = sum_{u,v<7, c<3} img[i][x+6-u][y+6-v][c] * filt[j][u][v][c]
template <int T>
__global__ void __launch_bounds__(T * T)
k_conv(const float *img, const float *filt, float *out, int n) {
    constexpr int TT = T + 6, KF = (147 + T * T - 1) / (T * T), KA = (TT + T - 1) / T;
    __shared__ float tile[TT][TT][3];
    __shared__ float fl[147];
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int gx = blockIdx.x, gy = blockIdx.y, zi = blockIdx.z / 3, zj = blockIdx.z % 3;
    const int64_t P = n + 6;
    for (int k = 0; k < KF; k++) {
        const int t = k * T * T + ly * T + lx;
        if (t < 147) fl[t] = filt[zj * 147 + t];
    }
    for (int a = 0; a < KA; a++)
        for (int b = 0; b < KA; b++) {
            const int r = a * T + ly, q = b * T + lx;
            const int64_t X = (int64_t)gy * T + r, Y = (int64_t)gx * T + q;
            if (r < TT && q < TT && X < P && Y < P)
                for (int c = 0; c < 3; c++) tile[r][q][c] = img[((zi * P + X) * P + Y) * 3 + c];
        }
    __syncthreads();
    const int x = gy * T + ly, y = gx * T + lx;
    if (x < n && y < n) {
        float acc = 0.f;
        for (int u = 0; u < 7; u++)
            for (int v = 0; v < 7; v++)
#pragma unroll
                for (int c = 0; c < 3; c++)
                    acc = __builtin_fmaf(tile[ly + 6 - u][lx + 6 - v][c], fl[(u * 7 + v) * 3 + c], acc);
        out[(((int64_t)zi * 3 + zj) * n + x) * n + y] = acc;
    }
}

// --------------------------------------------------------- barrier, empty
__global__ void k_barrier(float *out, int B) {
    for (int b = 0; b < B; b++) __syncthreads();
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)threadIdx.x;
}

__global__ void k_empty() {}

// ----------------------------------------------------------------- matmul
template <int T>
__global__ void __launch_bounds__(T * T)
k_mm_tiled(const float *A, const float *B, float *C, int n, int m, int l) {
    __shared__ float As[T][T];
    __shared__ float Bs[T][T + 1];
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int row = blockIdx.y * T + ly, col = blockIdx.x * T + lx;
    float acc = 0.f;
    const int KT = (m + T - 1) / T;
    for (int kt = 0; kt < KT; kt++) {
        const int ka = kt * T + lx, kb = kt * T + ly;
        As[ly][lx] = (row < n && ka < m) ? A[(int64_t)row * m + ka] : 0.f;
        Bs[ly][lx] = (kb < m && col < l) ? B[(int64_t)kb * l + col] : 0.f;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < T; kk++) acc = __builtin_fmaf(As[ly][kk], Bs[kk][lx], acc);
        __syncthreads();
    }
    if (row < n && col < l) C[(int64_t)row * l + col] = acc;
}

__global__ void k_mm_naive(const float *A, const float *B, float *C, int n,
                           int m, int l) {
    const int row = blockIdx.y * blockDim.y + threadIdx.y;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (row < n && col < l) {
        float acc = 0.f;
        for (int k = 0; k < m; k++)
            acc = __builtin_fmaf(A[(int64_t)row * m + k], B[(int64_t)k * l + col], acc);
        C[(int64_t)row * l + col] = acc;
    }
}

// -------------------------------------------------------------- transpose
template <int T>
__global__ void __launch_bounds__(T * T)
k_tr_tiled(const float *in, float *out, int n) {
    __shared__ float tile[T][T + 1];
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int r = blockIdx.y * T + ly, c = blockIdx.x * T + lx;
    if (r < n && c < n) tile[ly][lx] = in[(int64_t)r * n + c];
    __syncthreads();
    const int r2 = blockIdx.x * T + ly, c2 = blockIdx.y * T + lx;
    if (r2 < n && c2 < n) out[(int64_t)r2 * n + c2] = tile[lx][ly];
}

// writes coalesced: out[r][c] = in[c][r]
__global__ void k_tr_naive_wc(const float *in, float *out, int n) {
    const int r = blockIdx.y * blockDim.y + threadIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n && c < n) out[(int64_t)r * n + c] = in[(int64_t)c * n + r];
}

// reads coalesced: out[c][r] = in[r][c]
__global__ void k_tr_naive_rc(const float *in, float *out, int n) {
    const int r = blockIdx.y * blockDim.y + threadIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n && c < n) out[(int64_t)c * n + r] = in[(int64_t)r * n + c];
}

// ---------------------------------------------------------------- stencil
// Interior point (i, j) reads input cell (i+1, j+1) of the (n+2)^2 array;
// the tile and its four halo edges go through LDS.
template <typename T, int TS>
__global__ void __launch_bounds__(TS * TS)
k_stencil(const T *u, T *out, int n, T h2) {
    __shared__ T s[TS + 2][TS + 2];
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int i = blockIdx.y * TS + ly, j = blockIdx.x * TS + lx;
    const int64_t P = n + 2;
    const bool in = i < n && j < n;
    if (in) s[ly + 1][lx + 1] = u[(i + 1) * P + j + 1];
    if (ly == 0 && j < n) s[0][lx + 1] = u[i * P + j + 1];
    if (ly == TS - 1 && in) s[TS + 1][lx + 1] = u[(i + 2) * P + j + 1];
    if (ly < TS - 1 && i == n - 1 && j < n) s[ly + 2][lx + 1] = u[(i + 2) * P + j + 1];
    if (lx == 0 && i < n) s[ly + 1][0] = u[(i + 1) * P + j];
    if (lx == TS - 1 && in) s[ly + 1][TS + 1] = u[(i + 1) * P + j + 2];
    if (lx < TS - 1 && j == n - 1 && i < n) s[ly + 1][lx + 2] = u[(i + 1) * P + j + 2];
    __syncthreads();
    if (in) {
        const T c = s[ly + 1][lx + 1];
        const T r = (((s[ly][lx + 1] + s[ly + 2][lx + 1]) + s[ly + 1][lx]) +
                     s[ly + 1][lx + 2]) + h2 * (c * c);
        out[(int64_t)i * n + j] = (T)0.25 * r;
    }
}

// ------------------------------------------------------------------ nbody
// positions pos[c + 3 i]; blocks of G positions staged through LDS.  The
// terms of one block are summed into a partial, which is then added to the
// running total: an fp32 sum over N terms in two levels, G then N/G long.
__global__ void k_nbody(const float *__restrict__ pos, float *__restrict__ out, int N) {
    extern __shared__ float sh[];
    const int G = blockDim.x, l = threadIdx.x;
    const int i = blockIdx.x * G + l;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    if (i < N) {
        xi = pos[3 * (int64_t)i];
        yi = pos[3 * (int64_t)i + 1];
        zi = pos[3 * (int64_t)i + 2];
    }
    float acc = 0.f;
    const int GB = (N + G - 1) / G;
    for (int jb = 0; jb < GB; jb++) {
        const int j = jb * G + l;
        if (j < N) {
            sh[l] = pos[3 * (int64_t)j];
            sh[G + l] = pos[3 * (int64_t)j + 1];
            sh[2 * G + l] = pos[3 * (int64_t)j + 2];
        }
        __syncthreads();
        const int lim = N - jb * G < G ? N - jb * G : G;
        float part = 0.f;
        for (int jj = 0; jj < lim; jj++) {
            const float dx = xi - sh[jj], dy = yi - sh[G + jj], dz = zi - sh[2 * G + jj];
            const float r2 = (dx * dx + dy * dy) + dz * dz;
            const float t = rsqrtf(r2);
            part += (jb * G + jj != i) ? t : 0.f;
        }
        acc += part;
        __syncthreads();
    }
    if (i < N) out[i] = acc;
}

// =============================================================== dispatch
static int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

int buffers(const pm_variant &v, size_t *bytes, uint32_t *role, uint32_t *nb) {
    const int64_t e = v.dtype == PM_F64 ? 8 : 4;
    *nb = 0;
    auto add = [&](int64_t b, uint32_t r) {
        bytes[*nb] = (size_t)b;
        role[*nb] = r;
        (*nb)++;
    };
    switch (v.family) {
    case PM_FAM_STREAM: {
        int64_t G = v.n[0] / v.wg[0];
        if (v.op == PM_STREAM_FILLED) {
            add(e * v.stride * v.n[0] * v.reps, 0);
            add(e * v.n[0], 1);
            break;
        }
        int64_t span = e * G * v.gstride * v.wg[0] * v.stride * v.reps * v.vec;
        if (v.op == PM_STREAM_LOAD) add(span, 0), add(e * v.n[0], 3);
        else if (v.op == PM_STREAM_AXPBY) add(span, 0), add(span, 0), add(span, 2);
        else if (v.op == PM_STREAM_STORE) add(span, 2);
        else if (v.op == PM_STREAM_COPY) add(span, 0), add(span, 2);
        else {
            for (int a = 0; a < 4; a++) add(span, 0);
            add(span, 2);
        }
        break;
    }
    case PM_FAM_LDS:
    case PM_FAM_BARRIER: add(4 * v.n[0] * v.wg[0], 1); break;
    case PM_FAM_FMA:
    case PM_FAM_ARITH:
    case PM_FAM_RSQRT: add(e * v.n[0], 0), add(e * v.n[0], 1); break;
    case PM_FAM_CONV: {
        int64_t P = v.n[0] + 6;
        add(4 * 9 * P * P, 0), add(4 * 441, 0), add(4 * 9 * v.n[0] * v.n[0], 1);
        break;
    }
    case PM_FAM_EMPTY: break;
    case PM_FAM_MATMUL:
        add(4 * v.n[0] * v.n[1], 0), add(4 * v.n[1] * v.n[2], 0), add(4 * v.n[0] * v.n[2], 1);
        break;
    case PM_FAM_TRANSPOSE: add(4 * v.n[0] * v.n[0], 0), add(4 * v.n[0] * v.n[0], 1); break;
    case PM_FAM_STENCIL: add(e * (v.n[0] + 2) * (v.n[0] + 2), 0), add(e * v.n[0] * v.n[0], 1); break;
    case PM_FAM_NBODY: add(4 * 3 * v.n[0], 0), add(4 * v.n[0], 1); break;
    default: return PM_EINVAL;
    }
    return PM_OK;
}

template <typename T, int VEC, bool NT>
static void launch_stream_nt(const pm_variant &v, void *const *b, hipStream_t s) {
    int64_t G = v.n[0] / v.wg[0];
    // the op's buffers (load 2, store 1, copy 2, axpby 3, add4 5); the
    // caller's array holds no more
    const int nb = v.op == PM_STREAM_STORE ? 1 : v.op == PM_STREAM_AXPBY ? 3
                 : v.op == PM_STREAM_ADD4 ? 5 : 2;
    T *p[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int i = 0; i < nb; i++) p[i] = (T *)b[i];
    T nan = (T)__builtin_nan("");
    dim3 gr((unsigned)G), bl(v.wg[0]);
    const int64_t st = v.stride, gst = v.gstride;
    switch (v.op) {
    case PM_STREAM_LOAD:
        hipLaunchKernelGGL((k_stream<T, VEC, PM_STREAM_LOAD, NT>), gr, bl, 0, s, p[0], p[1], p[2], p[3], p[4], G, st, gst, v.reps, nan);
        break;
    case PM_STREAM_STORE:
        hipLaunchKernelGGL((k_stream<T, VEC, PM_STREAM_STORE, NT>), gr, bl, 0, s, p[0], p[1], p[2], p[3], p[4], G, st, gst, v.reps, nan);
        break;
    case PM_STREAM_COPY:
        hipLaunchKernelGGL((k_stream<T, VEC, PM_STREAM_COPY, NT>), gr, bl, 0, s, p[0], p[1], p[2], p[3], p[4], G, st, gst, v.reps, nan);
        break;
    case PM_STREAM_AXPBY:
        hipLaunchKernelGGL((k_stream<T, VEC, PM_STREAM_AXPBY, NT>), gr, bl, 0, s, p[0], p[1], p[2], p[3], p[4], G, st, gst, v.reps, nan);
        break;
    default:
        hipLaunchKernelGGL((k_stream<T, VEC, PM_STREAM_ADD4, NT>), gr, bl, 0, s, p[0], p[1], p[2], p[3], p[4], G, st, gst, v.reps, nan);
    }
}

template <typename T, int VEC>
static void launch_stream_t(const pm_variant &v, void *const *b, hipStream_t s) {
    if (v.flags & PM_FLAG_STREAMING) launch_stream_nt<T, VEC, true>(v, b, s);
    else launch_stream_nt<T, VEC, false>(v, b, s);
}

template <typename T>
static void launch_fma_t(const pm_variant &v, void *const *b, hipStream_t s) {
    dim3 gr((unsigned)(v.n[0] / v.wg[0])), bl(v.wg[0]);
    const T *in = (const T *)b[0];
    T *out = (T *)b[1];
    switch (v.chains) {
    case 1: hipLaunchKernelGGL((k_fma<T, 1>), gr, bl, 0, s, in, out, v.reps); break;
    case 2: hipLaunchKernelGGL((k_fma<T, 2>), gr, bl, 0, s, in, out, v.reps); break;
    case 4: hipLaunchKernelGGL((k_fma<T, 4>), gr, bl, 0, s, in, out, v.reps); break;
    case 8: hipLaunchKernelGGL((k_fma<T, 8>), gr, bl, 0, s, in, out, v.reps); break;
    default: hipLaunchKernelGGL((k_fma<T, 16>), gr, bl, 0, s, in, out, v.reps); break;
    }
}

template <typename T, int OP>
static void launch_arith_t(const pm_variant &v, void *const *b, hipStream_t s) {
    dim3 gr((unsigned)(v.n[0] / v.wg[0])), bl(v.wg[0]);
    const T *in = (const T *)b[0];
    T *out = (T *)b[1];
    switch (v.chains) {
    case 1: hipLaunchKernelGGL((k_arith<T, 1, OP>), gr, bl, 0, s, in, out, v.reps); break;
    case 2: hipLaunchKernelGGL((k_arith<T, 2, OP>), gr, bl, 0, s, in, out, v.reps); break;
    case 4: hipLaunchKernelGGL((k_arith<T, 4, OP>), gr, bl, 0, s, in, out, v.reps); break;
    default: hipLaunchKernelGGL((k_arith<T, 8, OP>), gr, bl, 0, s, in, out, v.reps); break;
    }
}

template <typename T>
static void launch_stencil_t(const pm_variant &v, void *const *b, hipStream_t s) {
    int n = (int)v.n[0], T_ = v.tile;
    T h2 = (T)(1.0 / ((double)(n + 1) * (double)(n + 1)));
    dim3 gr((unsigned)cdiv64(n, T_), (unsigned)cdiv64(n, T_)), bl(T_, T_);
    const T *u = (const T *)b[0];
    T *o = (T *)b[1];
    if (T_ == 8) hipLaunchKernelGGL((k_stencil<T, 8>), gr, bl, 0, s, u, o, n, h2);
    else if (T_ == 16) hipLaunchKernelGGL((k_stencil<T, 16>), gr, bl, 0, s, u, o, n, h2);
    else hipLaunchKernelGGL((k_stencil<T, 32>), gr, bl, 0, s, u, o, n, h2);
}

// Assumes v has passed the descriptor checks and the buffers their sizes.
int launch(const pm_variant &v, void *const *b, hipStream_t s) {
    switch (v.family) {
    case PM_FAM_STREAM:
        if (v.op == PM_STREAM_FILLED) {
            int64_t G = v.n[0] / v.wg[0];
            dim3 gr((unsigned)G), bl(v.wg[0]);
            const int c = v.chains ? v.chains : v.stride;
            if (v.dtype == PM_F64)
                hipLaunchKernelGGL(k_filled<double>, gr, bl, 0, s, (const double *)b[0], (double *)b[1], G, v.reps, v.stride, c);
            else
                hipLaunchKernelGGL(k_filled<float>, gr, bl, 0, s, (const float *)b[0], (float *)b[1], G, v.reps, v.stride, c);
        } else if (v.dtype == PM_F64) {
            if (v.vec == 1) launch_stream_t<double, 1>(v, b, s);
            else launch_stream_t<double, 2>(v, b, s);
        } else {
            if (v.vec == 1) launch_stream_t<float, 1>(v, b, s);
            else if (v.vec == 2) launch_stream_t<float, 2>(v, b, s);
            else launch_stream_t<float, 4>(v, b, s);
        }
        break;
    case PM_FAM_LDS: {
        dim3 gr((unsigned)v.n[0]), bl(v.wg[0]);
        size_t sh = (size_t)v.words * 4;
        if (v.op == PM_LDS_READ) hipLaunchKernelGGL(k_lds_read, gr, bl, sh, s, (float *)b[0], v.stride, v.reps, v.words);
        else hipLaunchKernelGGL(k_lds_write, gr, bl, sh, s, (float *)b[0], v.stride, v.reps, v.words);
        break;
    }
    case PM_FAM_FMA:
        if (v.dtype == PM_F64) launch_fma_t<double>(v, b, s);
        else launch_fma_t<float>(v, b, s);
        break;
    case PM_FAM_RSQRT: {
        dim3 gr((unsigned)(v.n[0] / v.wg[0])), bl(v.wg[0]);
        const float *in = (const float *)b[0];
        float *out = (float *)b[1];
        switch (v.chains) {
        case 1: hipLaunchKernelGGL(k_rsqrt<1>, gr, bl, 0, s, in, out, v.reps); break;
        case 2: hipLaunchKernelGGL(k_rsqrt<2>, gr, bl, 0, s, in, out, v.reps); break;
        case 4: hipLaunchKernelGGL(k_rsqrt<4>, gr, bl, 0, s, in, out, v.reps); break;
        default: hipLaunchKernelGGL(k_rsqrt<8>, gr, bl, 0, s, in, out, v.reps); break;
        }
        break;
    }
    case PM_FAM_BARRIER:
        hipLaunchKernelGGL(k_barrier, dim3((unsigned)v.n[0]), dim3(v.wg[0]), 0, s, (float *)b[0], v.reps);
        break;
    case PM_FAM_EMPTY: {
        int wy = v.wg[1] ? v.wg[1] : 1;
        hipLaunchKernelGGL(k_empty, dim3((unsigned)cdiv64(v.n[0], v.wg[0]), (unsigned)cdiv64(v.n[0], wy)), dim3(v.wg[0], wy), 0, s);
        break;
    }
    case PM_FAM_MATMUL: {
        int n = (int)v.n[0], m = (int)v.n[1], l = (int)v.n[2], T = v.tile;
        dim3 gr((unsigned)cdiv64(l, T), (unsigned)cdiv64(n, T)), bl(T, T);
        const float *A = (const float *)b[0], *B = (const float *)b[1];
        float *C = (float *)b[2];
        if (v.op == PM_MATMUL_NAIVE) hipLaunchKernelGGL(k_mm_naive, gr, bl, 0, s, A, B, C, n, m, l);
        else if (T == 8) hipLaunchKernelGGL(k_mm_tiled<8>, gr, bl, 0, s, A, B, C, n, m, l);
        else if (T == 16) hipLaunchKernelGGL(k_mm_tiled<16>, gr, bl, 0, s, A, B, C, n, m, l);
        else hipLaunchKernelGGL(k_mm_tiled<32>, gr, bl, 0, s, A, B, C, n, m, l);
        break;
    }
    case PM_FAM_TRANSPOSE: {
        int n = (int)v.n[0], T = v.tile;
        dim3 gr((unsigned)cdiv64(n, T), (unsigned)cdiv64(n, T)), bl(T, T);
        const float *in = (const float *)b[0];
        float *out = (float *)b[1];
        if (v.op == PM_TRANSPOSE_NAIVE_WC) hipLaunchKernelGGL(k_tr_naive_wc, gr, bl, 0, s, in, out, n);
        else if (v.op == PM_TRANSPOSE_NAIVE_RC) hipLaunchKernelGGL(k_tr_naive_rc, gr, bl, 0, s, in, out, n);
        else if (T == 8) hipLaunchKernelGGL(k_tr_tiled<8>, gr, bl, 0, s, in, out, n);
        else if (T == 16) hipLaunchKernelGGL(k_tr_tiled<16>, gr, bl, 0, s, in, out, n);
        else hipLaunchKernelGGL(k_tr_tiled<32>, gr, bl, 0, s, in, out, n);
        break;
    }
    case PM_FAM_STENCIL:
        if (v.dtype == PM_F64) launch_stencil_t<double>(v, b, s);
        else launch_stencil_t<float>(v, b, s);
        break;
    case PM_FAM_ARITH:
        if (v.dtype == PM_F64) {
            if (v.op == PM_ARITH_DIV) launch_arith_t<double, PM_ARITH_DIV>(v, b, s);
            else launch_arith_t<double, PM_ARITH_EXP>(v, b, s);
        } else {
            if (v.op == PM_ARITH_DIV) launch_arith_t<float, PM_ARITH_DIV>(v, b, s);
            else launch_arith_t<float, PM_ARITH_EXP>(v, b, s);
        }
        break;
    case PM_FAM_CONV: {
        int n = (int)v.n[0], T = v.tile;
        dim3 gr((unsigned)cdiv64(n, T), (unsigned)cdiv64(n, T), 9), bl(T, T);
        const float *img = (const float *)b[0], *fl = (const float *)b[1];
        float *o = (float *)b[2];
        if (T == 8) hipLaunchKernelGGL(k_conv<8>, gr, bl, 0, s, img, fl, o, n);
        else hipLaunchKernelGGL(k_conv<16>, gr, bl, 0, s, img, fl, o, n);
        break;
    }
    case PM_FAM_NBODY: {
        int N = (int)v.n[0], G = v.wg[0];
        hipLaunchKernelGGL(k_nbody, dim3((unsigned)cdiv64(N, G)), dim3(G), (size_t)12 * G, s, (const float *)b[0], (float *)b[1], N);
        break;
    }
    default: return PM_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}

}  // namespace pm
