"""Plain references of every kernel family's output.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Each function takes the input arrays (NumPy, the exact bytes uploaded to the
device) and returns the expected output array.  The kernels' arithmetic is
stated in their docstrings; where a kernel's result is exact (data movement,
sums in a fixed order in the kernel's own precision, single-rounding FMA
chains) the reference computes it in that precision in the same order;
otherwise (matmul, n-body, rsqrt chains) in float64.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import count as _count


def _np(dt):
    return np.float32 if dt == "f32" else np.float64


def stream_elements(v):
    """Flat element indices touched by a stream variant, in the order
    (u, g, l, component): index = vec*(((g*gs)*wg + l)*s + u*G*gs*wg*s) + c."""
    N, wg, s, gs, vec, U = (v["n"], v["wg"], v["s"], v["gs"], v["vec"],
                            v["U"])
    G = N // wg
    g = np.arange(G, dtype=np.int64)[:, None]
    l = np.arange(wg, dtype=np.int64)[None, :]
    base = ((g * gs) * wg + l) * s
    out = []
    for u in range(U):
        e = vec * (base + u * G * gs * wg * s)
        out.append((e[..., None] + np.arange(vec)).reshape(-1))
    return np.concatenate(out)


def stream_span(v):
    N, wg = v["n"], v["wg"]
    G = N // wg
    if v["op"] == "filled":
        return v["s"] * G * wg * v["U"]
    return G * v["gs"] * wg * v["s"] * v["U"] * v["vec"]


def stream_store(v, x0):
    """store: x[e] = (dtype)(e) at every touched element e; other elements
    keep their previous content."""
    x = x0.copy()
    e = stream_elements(v)
    x[e] = e.astype(x.dtype)
    return x


def stream_copy(v, x, y0):
    """copy: y[e] = x[e] at touched elements."""
    y = y0.copy()
    e = stream_elements(v)
    y[e] = x[e]
    return y


def stream_add4(v, a, b, c, d, o0):
    """add4: o[e] = (a[e] + b[e]) + (c[e] + d[e]) in the kernel dtype."""
    o = o0.copy()
    e = stream_elements(v)
    o[e] = (a[e] + b[e]) + (c[e] + d[e])
    return o


def stream_axpby(v, x, y, o0):
    """axpby: o[e] = 0.75 * x[e] + (-1.25) * y[e] in the kernel dtype."""
    o = o0.copy()
    e = stream_elements(v)
    t = x.dtype.type
    o[e] = t(0.75) * x[e] + t(-1.25) * y[e]
    return o


def stream_filled(v, x):
    """filled (lane stride s, c = v["c"] cells read of every s, c = s when
    absent): work-item i, for u = 0..U-1 and j = i + u*N, sums the cells
    x[s*j .. s*j+c-1] left to right, ((x0 + x1) + x2) + ..., and adds that
    to a running sum started at 0 (in the kernel dtype)."""
    N, U, s = v["n"], v["U"], v["s"]
    c = v.get("c", s)
    acc = np.zeros(N, dtype=x.dtype)
    i = np.arange(N, dtype=np.int64)
    for u in range(U):
        j = i + u * N
        t = x[s * j]
        for q in range(1, c):
            t = t + x[s * j + q]
        acc = acc + t
    return acc


def lds_out(v):
    """lds read: lane l of every group sums, from 0, the R words
    lds[(l*b + r) mod W] (r = 0..R-1) of an LDS array initialised with
    lds[a] = a, in fp32.  write: every lane writes lds[(l*b + r) mod W] = a
    for r = 0..R-1, then reads back lds[(l*b) mod W], which holds that
    address as a float."""
    G, wg, b, R, W = v["groups"], v["wg"], v["b"], v["R"], v["W"]
    l = np.arange(wg, dtype=np.int64)
    if v["op"] == "read":
        acc = np.zeros(wg, dtype=np.float32)
        for r in range(R):
            acc = acc + ((l * b + r) % W).astype(np.float32)
    else:
        acc = ((l * b) % W).astype(np.float32)
    return np.tile(acc, G)


def fma_chain(v, x):
    """fma: K chains start at a = in[i]; F/K rounds of c_k = fma(c_k, a,
    (k+1)/64); out[i] = ((c_0 + c_1) + ...) + c_{K-1}.  Computed with the C
    library's single-rounding fmaf / fma."""
    L = _count.lib()
    n = x.shape[0]
    out = np.empty_like(x)
    if x.dtype == np.float32:
        P = ctypes.POINTER(ctypes.c_float)
        L.oracle_fma_chain_f32(x.ctypes.data_as(P), out.ctypes.data_as(P), n,
                               v["F"], v["K"])
    else:
        P = ctypes.POINTER(ctypes.c_double)
        L.oracle_fma_chain_f64(x.ctypes.data_as(P), out.ctypes.data_as(P), n,
                               v["F"], v["K"])
    return out


def rsqrt_chain(v, x):
    """rsqrt: K chains y_k = a; F/K rounds of y_k = 1/sqrt(y_k*y_k + (k+1));
    out = sum of chains left to right.  float64 reference."""
    a = x.astype(np.float64)
    K, F = v["K"], v["F"]
    ys = [a.copy() for _ in range(K)]
    for _ in range(F // K):
        for k in range(K):
            ys[k] = 1.0 / np.sqrt(ys[k] * ys[k] + (k + 1))
    s = ys[0]
    for k in range(1, K):
        s = s + ys[k]
    return s


def div_chain(v, x):
    """arith div: K chains y_k = a; F/K rounds of y_k = (k+1) / (y_k*y_k + 1)
    in the kernel dtype (every step one IEEE rounding); out = sum of chains
    left to right."""
    t = x.dtype.type
    K, F = v["K"], v["F"]
    ys = [x.copy() for _ in range(K)]
    for _ in range(F // K):
        for k in range(K):
            ys[k] = t(k + 1) / (ys[k] * ys[k] + t(1))
    s = ys[0]
    for k in range(1, K):
        s = s + ys[k]
    return s


def exp_chain(v, x):
    """arith exp: K chains y_k = a; F/K rounds of y_k = exp(-(y_k*y_k));
    out = sum of chains.  float64 reference."""
    a = x.astype(np.float64)
    K, F = v["K"], v["F"]
    ys = [a.copy() for _ in range(K)]
    for _ in range(F // K):
        for k in range(K):
            ys[k] = np.exp(-(ys[k] * ys[k]))
    s = ys[0]
    for k in range(1, K):
        s = s + ys[k]
    return s


def conv(img, filt, n):
    """Three 7x7 filters over three RGB images (n+6)^2 x 3, channel fastest:
    r[i][j][x][y] = sum over u, v < 7 and c < 3 of
    img[i][x+6-u][y+6-v][c] * filt[j][u][v][c], in float64.  Returns
    (r, sum of |terms|) with shape (3, 3, n, n)."""
    P = n + 6
    I = img.reshape(3, P, P, 3).astype(np.float64)
    Fw = filt.reshape(3, 7, 7, 3).astype(np.float64)
    r = np.zeros((3, 3, n, n))
    a = np.zeros((3, 3, n, n))
    for u in range(7):
        for v in range(7):
            win = I[:, 6 - u:6 - u + n, 6 - v:6 - v + n, :]  # (3, n, n, 3)
            r += np.einsum("ixyc,jc->ijxy", win, Fw[:, u, v, :])
            a += np.einsum("ixyc,jc->ijxy", np.abs(win), np.abs(Fw[:, u, v, :]))
    return r, a


def conv_at(img, filt, n, idx):
    """The convolution of `conv` at sampled outputs only: idx is an array of
    (image i, filter j, x, y) rows; returns (r, sum of |terms|) for them,
    each the 147-term sum over u, v < 7 and c < 3 of
    img[i][x+6-u][y+6-v][c] * filt[j][u][v][c] in float64."""
    P = n + 6
    I = img.reshape(3, P, P, 3).astype(np.float64)
    Fw = filt.reshape(3, 7, 7, 3).astype(np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    r = np.zeros(len(idx))
    a = np.zeros(len(idx))
    for t, (i, j, x, y) in enumerate(idx):
        win = I[i, x:x + 7, y:y + 7, :][::-1, ::-1, :]  # win[u, v] = img[x+6-u, y+6-v]
        r[t] = (win * Fw[j]).sum()
        a[t] = (np.abs(win) * np.abs(Fw[j])).sum()
    return r, a


def barrier_out(v):
    """barrier: each work-item stores its local id as a float."""
    return np.tile(np.arange(v["wg"], dtype=np.float32), v["groups"])


def matmul(A, B):
    """C = A B in float64 (A: n x m, B: m x l, row-major)."""
    return A.astype(np.float64) @ B.astype(np.float64)


def matmul_abs(A, B):
    """sum_k |a_ik| |b_kj|, the scale of the matmul error bound."""
    return np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))


def transpose(A):
    return np.ascontiguousarray(A.T)


def stencil(u, n, dt):
    """5-point stencil with a quadratic source term on the (n+2)^2 input
    (halo ring included), output n x n, in the kernel dtype:
    out = 0.25 * ((((N + S) + W) + E) + h2 * (c * c)), h2 = 1/(n+1)^2."""
    t = _np(dt)
    u = u.reshape(n + 2, n + 2)
    h2 = t(1.0 / ((n + 1.0) * (n + 1.0)))
    c = u[1:-1, 1:-1]
    N = u[:-2, 1:-1]
    S = u[2:, 1:-1]
    W = u[1:-1, :-2]
    E = u[1:-1, 2:]
    out = t(0.25) * ((((N + S) + W) + E) + h2 * (c * c))
    return out.astype(t)


def stencil_abs(u, n, dt):
    """Magnitude scale of the stencil terms, for a rounding-error bound."""
    u = np.abs(u.reshape(n + 2, n + 2).astype(np.float64))
    h2 = 1.0 / ((n + 1.0) * (n + 1.0))
    return 0.25 * (u[:-2, 1:-1] + u[2:, 1:-1] + u[1:-1, :-2] + u[1:-1, 2:]
                   + h2 * u[1:-1, 1:-1] ** 2)


def nbody(pos, idx=None):
    """pos: 3 x N column-major (pos[c + 3 i]).  out[i] = sum over j != i of
    1 / |x_i - x_j|, float64.  Returns (out, sum of |terms|) for the rows
    `idx` (all rows by default)."""
    P = pos.reshape(-1, 3).astype(np.float64)
    N = P.shape[0]
    rows = np.arange(N) if idx is None else np.asarray(idx)
    out = np.empty(len(rows))
    for t, i in enumerate(rows):
        d = P - P[i]
        r = np.sqrt((d * d).sum(axis=1))
        r[i] = np.inf
        out[t] = (1.0 / r).sum()
    return out, out.copy()
