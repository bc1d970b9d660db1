"""Derived features, the relative-error fit (Sec. 4.3) and the error metric
(Sec. 5) in plain NumPy float64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Feature sets (projections of the count dict of oracle.count.count):

  p3    the three-feature plain model: [global load+store bytes, fp32 FMAs,
        work-groups]
  p12   [const 1, work-groups, barriers summed over work-items,
         fp32 add+mul (an FMA counts once for each), fp64 add+mul,
         special+div+exp (both dtypes), LDS bytes (loads+stores),
         global-load bytes in classes 0, 1, 2/2, 3/3, 4/4,
         global-store bytes in those classes,
         global-load bytes in the other classes (k<q, and every '>4' bin),
         global-store bytes in the other classes,
         min(stride-1 load bytes, stride-1 store bytes)]
  full  the paper's own property list (Sec. 2): one column per global
        (direction, size, class) count, per LDS (direction, size), per flop
        (kind, dtype) with an FMA counted as one add and one mul, barriers,
        work-groups, const 1, and min(loads, stores) per (size, class)
  ext   full and the extensions the paper names as future work (Sec. 6):
        arithmetic instructions and global bytes per resident work-item,
        min(arithmetic instructions, global bytes)
  bank  ext with its six LDS counts replaced by the LDS counts per
        (direction, size, bank-stride bin) -- the binning of the LDS stride
        Sec. 6.2 proposes (bins b0 = broadcast, b1 = odd stride, b2 ... b32
        = the power of two in the stride, 32 and more together)
"""
from __future__ import annotations

import math

import numpy as np

CLASSES = ["0", "1", "1/2", "2/2", "1/3", "2/3", "3/3", "1/4", "2/4", "3/4",
           "4/4", "1/>4", "2/>4", "3/>4", "4/>4"]
FULL_USE = {"0", "1", "2/2", "3/3", "4/4"}
SIZES = [4, 8, 16]


def _g(c, key):
    return c.get(key, 0)


def _gbytes(c, d, pred):
    t = 0
    for sz in SIZES:
        for cl in CLASSES:
            if pred(cl):
                t += sz * _g(c, "%s.%d.%s" % (d, sz, cl))
    return t


def features_p3(c):
    gb = _gbytes(c, "gld", lambda cl: True) + _gbytes(c, "gst", lambda cl: True)
    return [float(gb), float(_g(c, "fma.f32")), float(_g(c, "wg"))]


def features_p12(c):
    f32 = _g(c, "add.f32") + _g(c, "mul.f32") + 2 * _g(c, "fma.f32")
    f64 = _g(c, "add.f64") + _g(c, "mul.f64") + 2 * _g(c, "fma.f64")
    spec = sum(_g(c, "%s.%s" % (k, d)) for k in ("spec", "div", "exp")
               for d in ("f32", "f64"))
    ldsb = sum(sz * (_g(c, "lld.%d" % sz) + _g(c, "lst.%d" % sz))
               for sz in SIZES)
    full = lambda cl: cl in FULL_USE  # noqa: E731
    part = lambda cl: cl not in FULL_USE  # noqa: E731
    s1 = lambda cl: cl == "1"  # noqa: E731
    return [1.0, float(_g(c, "wg")), float(_g(c, "bar.wi")), float(f32),
            float(f64), float(spec), float(ldsb),
            float(_gbytes(c, "gld", full)), float(_gbytes(c, "gst", full)),
            float(_gbytes(c, "gld", part)), float(_gbytes(c, "gst", part)),
            float(min(_gbytes(c, "gld", s1), _gbytes(c, "gst", s1)))]


def full_names():
    names = []
    for d in ("gld", "gst"):
        for sz in SIZES:
            for cl in CLASSES:
                names.append("%s.%d.%s" % (d, sz, cl))
    for d in ("lld", "lst"):
        for sz in SIZES:
            names.append("%s.%d" % (d, sz))
    for k in ("add", "mul", "div", "exp", "spec"):
        for dt in ("f32", "f64"):
            names.append("%s.%s" % (k, dt))
    names += ["bar.wi", "wg", "const"]
    for sz in SIZES:
        for cl in CLASSES:
            names.append("min.%d.%s" % (sz, cl))
    return names


def features_full(c):
    out = []
    for d in ("gld", "gst"):
        for sz in SIZES:
            for cl in CLASSES:
                out.append(float(_g(c, "%s.%d.%s" % (d, sz, cl))))
    for d in ("lld", "lst"):
        for sz in SIZES:
            out.append(float(_g(c, "%s.%d" % (d, sz))))
    for k in ("add", "mul", "div", "exp", "spec"):
        for dt in ("f32", "f64"):
            x = _g(c, "%s.%s" % (k, dt))
            if k in ("add", "mul"):
                x += _g(c, "fma.%s" % dt)
            out.append(float(x))
    out += [float(_g(c, "bar.wi")), float(_g(c, "wg")), 1.0]
    for sz in SIZES:
        for cl in CLASSES:
            out.append(float(min(_g(c, "gld.%d.%s" % (sz, cl)),
                                 _g(c, "gst.%d.%s" % (sz, cl)))))
    return out


RESIDENT_WI = 256 * 2048  # work-items the GPU holds at once


def features_ext(c):
    """The paper's list plus its named extensions (Sec. 6): arithmetic
    instructions and global bytes per resident work-item, and
    min(arithmetic instructions, global bytes)."""
    ops = sum(_g(c, "%s.%s" % (k, dt)) for k in ("add", "mul", "div", "exp", "spec", "fma")
              for dt in ("f32", "f64"))
    gb = _gbytes(c, "gld", lambda cl: True) + _gbytes(c, "gst", lambda cl: True)
    wi = min(_g(c, "wi"), RESIDENT_WI)
    return features_full(c) + [ops / wi if wi else 0.0, gb / wi if wi else 0.0,
                               float(min(ops, gb))]


BANK_BINS = ["b0", "b1", "b2", "b4", "b8", "b16", "b32"]


def features_bank(c):
    """features_ext with the 6 LDS counts (after the 90 global ones) replaced
    by the 42 LDS counts by bank-stride bin."""
    e = features_ext(c)
    binned = [float(_g(c, "%s.%d.%s" % (d, sz, b)))
              for d in ("lld", "lst") for sz in SIZES for b in BANK_BINS]
    return e[:90] + binned + e[96:]


FEATURES = {"p3": features_p3, "p12": features_p12, "full": features_full,
            "ext": features_ext, "bank": features_bank}


def feature_matrix(counts, proj):
    f = FEATURES[proj]
    return np.array([f(c) for c in counts], dtype=np.float64)


def fit(P, T):
    """Weights minimising sum_j (1 - sum_i a_i P_ji / T_j)^2 (Sec. 4.3):
    each row of the property matrix is divided by its measured time and the
    least-squares problem A a = 1 is solved (numpy.linalg.lstsq, minimum
    norm).  All-zero columns are left out and get weight 0."""
    P = np.asarray(P, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    A = P / T[:, None]
    keep = np.any(A != 0.0, axis=0)
    alpha = np.zeros(P.shape[1])
    sol, _, rank, sv = np.linalg.lstsq(A[:, keep], np.ones(len(T)), rcond=None)
    alpha[keep] = sol
    return alpha, int(rank)


def predict(P, alpha):
    return np.asarray(P, dtype=np.float64) @ np.asarray(alpha, np.float64)


def rel_errors(pred, actual):
    """|predicted - actual| / actual (Sec. 5)."""
    pred = np.asarray(pred, dtype=np.float64)
    actual = np.asarray(actual, dtype=np.float64)
    return np.abs(pred - actual) / actual


def geomean(x, floor=1e-12):
    """Geometric mean; zero entries are floored at `floor`."""
    x = np.maximum(np.asarray(x, dtype=np.float64), floor)
    return float(math.exp(np.mean(np.log(x))))
