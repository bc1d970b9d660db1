"""Python binding of libpm (include/pm.h): argument marshalling only.

Every step of counting, prediction and measurement runs in libpm's HIP
kernels (and its FP64 host fit); this module converts variant dicts (see
synth/inputs.py for the parameter names) to `pm_variant` structs and
passes device pointers of PyTorch tensors.  Importing fails loudly when
libpm.so has not been built (python -m paper_1604_04997_amd.build).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpm.so")

PM_NCOUNT = 154
PM_NFEAT_MAX = 200
PM_MAXBUF = 8
PM_BATCH_MAX = 65536
PM_NOALLOC_MAX_VARIANTS = 1024
PROJ = {"p3": 0, "p12": 1, "full": 2, "ext": 3, "bank": 4}
NFEAT = {"p3": 3, "p12": 12, "full": 154, "ext": 157, "bank": 193}

FAMILY = {"stream": 0, "lds": 1, "fma": 2, "rsqrt": 3, "barrier": 4,
          "empty": 5, "matmul": 6, "transpose": 7, "stencil": 8, "nbody": 9,
          "arith": 10, "conv": 11}
OPS = {
    "stream": {"load": 0, "store": 1, "copy": 2, "add4": 3, "filled": 4,
               "axpby": 5},
    "arith": {"div": 0, "exp": 1},
    "lds": {"read": 0, "write": 1},
    "matmul": {"tiled": 0, "naive": 1},
    "transpose": {"tiled": 0, "naive_wc": 1, "naive_rc": 2},
}
STATUS = {0: "PM_OK", -1: "PM_EINVAL", -2: "PM_ENOMEM", -3: "PM_EDEVICE",
          -4: "PM_ERANK", -5: "PM_EOVERFLOW", -6: "PM_ETIMEDOUT",
          -7: "PM_EBUSY"}


class Variant(ctypes.Structure):
    _fields_ = [("family", ctypes.c_uint32), ("dtype", ctypes.c_uint32),
                ("op", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("n", ctypes.c_int64 * 3), ("wg", ctypes.c_int32 * 2),
                ("tile", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("gstride", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("reps", ctypes.c_int32), ("chains", ctypes.c_int32),
                ("words", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class Counts(ctypes.Structure):
    _fields_ = [("c", ctypes.c_int64 * PM_NCOUNT)]


class Model(ctypes.Structure):
    _fields_ = [("nfeat", ctypes.c_uint32), ("proj", ctypes.c_uint32),
                ("alpha", ctypes.c_double * PM_NFEAT_MAX)]


class Schedule(ctypes.Structure):
    _fields_ = [("inblock_items", ctypes.c_int64), ("fused_items", ctypes.c_int64),
                ("tail_wgs_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32)]


QPOLY_MAXPERIOD = 64
QPOLY_DEGREE = 3


class QPoly(ctypes.Structure):
    _fields_ = [("base", Variant), ("fields", ctypes.c_uint32), ("period", ctypes.c_int32),
                ("scale", ctypes.c_int64), ("x0", ctypes.c_int64),
                ("coef", ctypes.c_int64 * PM_NCOUNT * (QPOLY_DEGREE + 1) * QPOLY_MAXPERIOD)]


class PMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


_lib = None


def lib():
    """Load libpm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpm.so not built: run "
                              "`python -m paper_1604_04997_amd.build`")
        # torch's wheel ships a HIP runtime under the same soname as the one
        # libpm.so links: whichever loads first serves the whole process, and
        # torch does not run on another release's.  Load torch's first (device
        # buffers and streams come from torch); without torch, ROCm's serves.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        sigs = {
            "pm_create": (ctypes.c_int, [P(vp), ctypes.c_int, ctypes.c_size_t]),
            "pm_destroy": (None, [vp]),
            "pm_last_error": (ctypes.c_char_p, []),
            "pm_count_name": (ctypes.c_int, [ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]),
            "pm_count": (ctypes.c_int, [vp, P(Variant), ctypes.c_size_t, P(Counts)]),
            "pm_predict": (ctypes.c_int, [vp, P(Model), P(Variant), ctypes.c_size_t, P(ctypes.c_double)]),
            "pm_count_device": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp, P(Model), vp, vp, vp]),
            "pm_count_device_noalloc": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp, P(Model), vp, vp, vp]),
            "pm_reserve": (ctypes.c_int, [vp, ctypes.c_size_t, ctypes.c_size_t]),
            "pm_qpoly_derive": (ctypes.c_int, [vp, P(Variant), ctypes.c_uint32, ctypes.c_int64,
                                               ctypes.c_int32, ctypes.c_int64, P(QPoly)]),
            "pm_qpoly_eval": (ctypes.c_int, [P(QPoly), ctypes.c_int64, P(Counts)]),
            "pm_qpoly_eval_many": (ctypes.c_int, [P(QPoly), P(ctypes.c_int64), ctypes.c_size_t,
                                                  P(Counts)]),
            "pm_bitmap_bytes": (ctypes.c_int, [P(Variant), P(ctypes.c_size_t)]),
            "pm_features": (ctypes.c_int, [P(Counts), ctypes.c_uint32, P(ctypes.c_double), P(ctypes.c_uint32)]),
            "pm_fit": (ctypes.c_int, [P(Counts), P(ctypes.c_double), ctypes.c_size_t, ctypes.c_uint32,
                                      P(Model), P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_uint32)]),
            "pm_buffers": (ctypes.c_int, [P(Variant), P(ctypes.c_size_t), P(ctypes.c_uint32), P(ctypes.c_uint32)]),
            "pm_launch": (ctypes.c_int, [vp, P(Variant), P(vp), P(ctypes.c_size_t), ctypes.c_uint32, vp]),
            "pm_measure": (ctypes.c_int, [vp, P(Variant), P(vp), P(ctypes.c_size_t), ctypes.c_uint32, vp,
                                          ctypes.c_int, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double)]),
            "pm_measure_until": (ctypes.c_int, [vp, P(Variant), P(vp), P(ctypes.c_size_t), ctypes.c_uint32, vp,
                                                ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                P(ctypes.c_double), P(ctypes.c_double),
                                                P(ctypes.c_int32), P(ctypes.c_uint32)]),
            "pm_launch_floor": (ctypes.c_int, [vp, vp, P(ctypes.c_double)]),
            "pm_count_host": (ctypes.c_int, [P(Variant), P(Counts), P(ctypes.c_int64)]),
            "pm_count_host_seq": (ctypes.c_int, [P(Variant), P(Counts), P(ctypes.c_int64)]),
            "pm_profile": (ctypes.c_int, [vp, ctypes.c_int]),
            "pm_profile_read": (ctypes.c_int, [vp, P(ctypes.c_double), P(ctypes.c_int)]),
            "pm_profile_sample": (ctypes.c_int, [vp, ctypes.c_int]),
            "pm_batch_stats": (ctypes.c_int, [vp, P(ctypes.c_int64)]),
            "pm_set_schedule": (ctypes.c_int, [vp, P(Schedule)]),
            "pm_get_schedule": (ctypes.c_int, [vp, P(Schedule)]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise PMError(rc, lib().pm_last_error().decode())


_names = None


def count_names():
    global _names
    if _names is None:
        buf = ctypes.create_string_buffer(32)
        out = []
        for i in range(PM_NCOUNT):
            _check(lib().pm_count_name(i, buf, 32))
            out.append(buf.value.decode())
        _names = out
    return _names


def variant_struct(d: dict) -> Variant:
    """Marshal a variant dict into a pm_variant."""
    v = Variant()
    fam = d["family"]
    v.family = FAMILY[fam]
    v.dtype = 1 if d.get("dtype", "f32") == "f64" else 0
    v.op = OPS.get(fam, {}).get(d.get("op"), 0)
    v.seed = int(d.get("seed", 0)) & ((1 << 64) - 1)
    v.flags = ((1 if d.get("bitmap") else 0) | (2 if d.get("enumerate") else 0)
               | (4 if d.get("streaming") else 0))
    if fam == "stream":
        v.n[0], v.wg[0] = d["n"], d["wg"]
        v.stride, v.gstride, v.vec, v.reps = d["s"], d.get("gs", 1), d.get("vec", 1), d.get("U", 1)
        if d.get("op") == "filled":
            v.chains = d.get("c", 0)  # cells read of every s (0: all s)
    elif fam == "lds":
        v.n[0], v.wg[0] = d["groups"], d["wg"]
        v.stride, v.reps, v.words = d["b"], d["R"], d["W"]
    elif fam in ("fma", "rsqrt", "arith"):
        v.n[0], v.wg[0], v.reps, v.chains = d["n"], d["wg"], d["F"], d["K"]
    elif fam == "barrier":
        v.n[0], v.wg[0], v.reps = d["groups"], d["wg"], d["B"]
    elif fam == "empty":
        v.n[0], v.wg[0], v.wg[1] = d["n"], d["wx"], d.get("wy", 1)
    elif fam == "matmul":
        v.n[0], v.n[1], v.n[2], v.tile = d["n"], d["m"], d["l"], d["T"]
    elif fam in ("transpose", "stencil", "conv"):
        v.n[0], v.tile = d["n"], d["T"]
    elif fam == "nbody":
        v.n[0], v.wg[0] = d["n"], d["wg"]
    return v


def variant_array(variants) -> ctypes.Array:
    arr = (Variant * len(variants))()
    for i, d in enumerate(variants):
        arr[i] = variant_struct(d)
    return arr


def counts_dict(c: Counts) -> dict:
    return {nm: int(x) for nm, x in zip(count_names(), c.c) if x}


def counts_numpy(arr) -> np.ndarray:
    return np.ctypeslib.as_array(arr).view(np.int64).reshape(len(arr), PM_NCOUNT) \
        if len(arr) else np.zeros((0, PM_NCOUNT), np.int64)


def model_struct(proj: str, alpha) -> Model:
    m = Model()
    m.proj = PROJ[proj]
    m.nfeat = NFEAT[proj]
    for i, a in enumerate(alpha):
        m.alpha[i] = float(a)
    return m


def model_alpha(m: Model) -> np.ndarray:
    return np.array(m.alpha[:m.nfeat], dtype=np.float64)


def features(counts: Counts, proj: str) -> np.ndarray:
    f = (ctypes.c_double * PM_NFEAT_MAX)()
    nf = ctypes.c_uint32()
    _check(lib().pm_features(ctypes.byref(counts), PROJ[proj], f, ctypes.byref(nf)))
    return np.array(f[:nf.value])


def fit(counts, T, proj: str):
    """Relative-error fit of Sec. 4.3 on the host in FP64.  counts: a ctypes
    Counts array; T: seconds.  Returns (Model, cond, resid, rank)."""
    n = len(counts)
    Tc = (ctypes.c_double * n)(*[float(t) for t in T])
    m = Model()
    cond = ctypes.c_double()
    resid = (ctypes.c_double * n)()
    rank = ctypes.c_uint32()
    _check(lib().pm_fit(counts, Tc, n, PROJ[proj], ctypes.byref(m),
                        ctypes.byref(cond), resid, ctypes.byref(rank)))
    return m, cond.value, np.array(resid[:]), rank.value


def qpoly_eval(qp: QPoly, x: int) -> Counts:
    """Counts of the quasi-polynomial at size x (host, O(1))."""
    c = Counts()
    _check(lib().pm_qpoly_eval(ctypes.byref(qp), int(x), ctypes.byref(c)))
    return c


def qpoly_eval_many(qp: QPoly, xs) -> ctypes.Array:
    """Counts of the quasi-polynomial at every size in xs (host)."""
    n = len(xs)
    xa = (ctypes.c_int64 * max(n, 1))(*[int(x) for x in xs])
    out = (Counts * max(n, 1))()
    _check(lib().pm_qpoly_eval_many(ctypes.byref(qp), xa, n, out))
    return out


def qpoly_sizes(d: dict, fields: int, scale: int, x: int) -> dict:
    """The variant dict with the size fields of `fields` set to scale * x
    (the variant a quasi-polynomial's value at x describes)."""
    keys = ["n", "m", "l"] if d["family"] == "matmul" else ["n"]
    out = dict(d)
    for i, k in enumerate(keys):
        if (fields >> i) & 1:
            out[k] = scale * x
    return out


def buffers(d: dict):
    """[(bytes, role)] of the variant's kernel buffers."""
    v = variant_struct(d)
    b = (ctypes.c_size_t * PM_MAXBUF)()
    r = (ctypes.c_uint32 * PM_MAXBUF)()
    nb = ctypes.c_uint32()
    _check(lib().pm_buffers(ctypes.byref(v), b, r, ctypes.byref(nb)))
    return [(int(b[i]), int(r[i])) for i in range(nb.value)]


def bitmap_bytes(d: dict) -> int:
    v = variant_struct(d)
    out = ctypes.c_size_t()
    _check(lib().pm_bitmap_bytes(ctypes.byref(v), ctypes.byref(out)))
    return out.value


def count_host(d: dict, with_footprints: bool = False, sequential: bool = False):
    """Test hook: the library's descriptor/count code run on the host
    (`sequential`: the one-pass descriptor expansion)."""
    v = variant_struct(d)
    c = Counts()
    foot = (ctypes.c_int64 * 12)()
    fn = lib().pm_count_host_seq if sequential else lib().pm_count_host
    _check(fn(ctypes.byref(v), ctypes.byref(c), foot))
    res = counts_dict(c)
    if with_footprints:
        for a in range(6):
            if foot[2 * a]:
                res["foot.F.%d" % a] = int(foot[2 * a])
                res["foot.fill.%d" % a] = int(foot[2 * a + 1])
    return res


class Context:
    """A libpm context on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().pm_create(ctypes.byref(self._h), device, hbm_budget))
        self.device = device

    def close(self):
        if self._h:
            lib().pm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def count_raw(self, variants):
        va = variants if isinstance(variants, ctypes.Array) else variant_array(variants)
        out = (Counts * len(va))()
        _check(lib().pm_count(self._h, va, len(va), out))
        return out

    def count(self, variants):
        """Count vectors of the variants as a list of {name: count}."""
        return [counts_dict(c) for c in self.count_raw(variants)]

    def predict(self, model: Model, variants) -> np.ndarray:
        va = variants if isinstance(variants, ctypes.Array) else variant_array(variants)
        t = (ctypes.c_double * len(va))()
        _check(lib().pm_predict(self._h, ctypes.byref(model), va, len(va), t))
        return np.array(t[:])

    PHASES = ("build", "gap", "tail")

    def profile(self, enable=True):
        """True / 1: events around every phase; 2: around the expansion
        kernel only (the lightest); False / 0: off."""
        _check(lib().pm_profile(self._h, int(enable)))

    def profile_sample(self, every: int):
        """Events on one batch in `every` of the timing window."""
        _check(lib().pm_profile_sample(self._h, int(every)))

    def profile_read(self):
        """({kernel: mean milliseconds}, batches) since profiling started."""
        ms = (ctypes.c_double * len(self.PHASES))()
        nb = ctypes.c_int()
        _check(lib().pm_profile_read(self._h, ms, ctypes.byref(nb)))
        return dict(zip(self.PHASES, ms[:])), nb.value

    def schedule(self) -> dict:
        """The batched counter's schedule (pm_get_schedule)."""
        sc = Schedule()
        _check(lib().pm_get_schedule(self._h, ctypes.byref(sc)))
        return {"inblock_items": sc.inblock_items, "fused_items": sc.fused_items,
                "tail_wgs_per_cu": sc.tail_wgs_per_cu}

    def set_schedule(self, **kw):
        """Change fields of the schedule (pm_set_schedule); returns the new one."""
        cur = self.schedule()
        unknown = set(kw) - set(cur)
        if unknown:
            raise KeyError("no schedule field %s" % sorted(unknown))
        cur.update(kw)
        sc = Schedule(cur["inblock_items"], cur["fused_items"], cur["tail_wgs_per_cu"], 0)
        _check(lib().pm_set_schedule(self._h, ctypes.byref(sc)))
        return self.schedule()

    def batch_stats(self) -> dict:
        st = (ctypes.c_int64 * 8)()
        _check(lib().pm_batch_stats(self._h, st))
        return {"chunks": st[0], "bitmap_words": st[1], "fill_segments": st[2],
                "handed_on": st[3], "bitmap_words_requested": st[4]}

    def reserve(self, nv: int, bitmap_bytes_: int):
        _check(lib().pm_reserve(self._h, nv, bitmap_bytes_))

    def count_device(self, d_variants_ptr, nv, d_counts_ptr, model, d_t_ptr,
                     d_status_ptr, stream_ptr):
        """Device-resident batched count (+ predict), asynchronous on the
        given stream; all pointers are device addresses (ints)."""
        _check(lib().pm_count_device(
            self._h, ctypes.c_void_p(d_variants_ptr), nv,
            ctypes.c_void_p(d_counts_ptr) if d_counts_ptr else None,
            ctypes.byref(model) if model is not None else None,
            ctypes.c_void_p(d_t_ptr) if d_t_ptr else None,
            ctypes.c_void_p(d_status_ptr), ctypes.c_void_p(stream_ptr)))

    def count_device_call(self, d_variants_ptr, nv, d_counts_ptr, model, d_t_ptr,
                          d_status_ptr, stream_ptr):
        """count_device with its arguments marshalled once: returns a
        function of no arguments that enqueues the same batch again (for a
        loop that repeats one batch on buffers that stay where they are)."""
        f = lib().pm_count_device
        args = (self._h, ctypes.c_void_p(d_variants_ptr), ctypes.c_size_t(nv),
                ctypes.c_void_p(d_counts_ptr) if d_counts_ptr else None,
                ctypes.byref(model) if model is not None else None,
                ctypes.c_void_p(d_t_ptr) if d_t_ptr else None,
                ctypes.c_void_p(d_status_ptr), ctypes.c_void_p(stream_ptr))

        def call(_keep=(model, args)):
            st = f(*args)
            if st:
                _check(st)
        return call

    def qpoly_derive(self, d: dict, fields: int = 1, scale: int = 1, period: int = 1,
                     x0: int = 1) -> QPoly:
        """pm_qpoly_derive: the counts of `d` with its size fields (bit 0 n,
        1 m, 2 l) set to scale * x, as quasi-polynomials in x derived by the
        batched counter."""
        qp = QPoly()
        v = variant_struct(d)
        _check(lib().pm_qpoly_derive(self._h, ctypes.byref(v), fields, scale, period, x0,
                                     ctypes.byref(qp)))
        return qp

    def count_device_noalloc(self, d_variants_ptr, nv, d_counts_ptr, model, d_t_ptr,
                             d_status_ptr, stream_ptr):
        """pm_count_device_noalloc: count_device with the library's fixed
        device array as working memory (no allocation)."""
        _check(lib().pm_count_device_noalloc(
            self._h, ctypes.c_void_p(d_variants_ptr), nv,
            ctypes.c_void_p(d_counts_ptr) if d_counts_ptr else None,
            ctypes.byref(model) if model is not None else None,
            ctypes.c_void_p(d_t_ptr) if d_t_ptr else None,
            ctypes.c_void_p(d_status_ptr), ctypes.c_void_p(stream_ptr)))

    def _bufs(self, tensors):
        n = len(tensors)
        ptrs = (ctypes.c_void_p * max(n, 1))(*[t.data_ptr() for t in tensors])
        sizes = (ctypes.c_size_t * max(n, 1))(*[t.numel() * t.element_size() for t in tensors])
        return ptrs, sizes, n

    @staticmethod
    def _stream(stream_ptr):
        """The given hipStream_t, else torch's current stream, so that kernels
        are ordered after the torch work that filled their buffers."""
        if stream_ptr is not None:
            return ctypes.c_void_p(stream_ptr)
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def launch(self, d: dict, tensors, stream_ptr=None):
        v = variant_struct(d)
        ptrs, sizes, n = self._bufs(tensors)
        _check(lib().pm_launch(self._h, ctypes.byref(v), ptrs, sizes, n,
                               self._stream(stream_ptr)))

    def measure(self, d: dict, tensors, warmup: int = 4, reps: int = 26,
                stream_ptr=None):
        """(min seconds, all rep times) of the variant's kernel (Sec. 4.2)."""
        v = variant_struct(d)
        ptrs, sizes, n = self._bufs(tensors)
        tr = (ctypes.c_double * reps)()
        tmin = ctypes.c_double()
        _check(lib().pm_measure(self._h, ctypes.byref(v), ptrs, sizes, n,
                                self._stream(stream_ptr), warmup, reps, tr,
                                ctypes.byref(tmin)))
        return tmin.value, list(tr[:])

    def launch_floor(self, stream_ptr=None) -> float:
        """Launch overhead in seconds: the empty kernel's minimum time
        (Sec. 4.2); the context keeps it for measure_until's floor check."""
        t = ctypes.c_double()
        _check(lib().pm_launch_floor(self._h, self._stream(stream_ptr), ctypes.byref(t)))
        return t.value

    def measure_until(self, d: dict, tensors, warmup: int = 4, reps: int = 26,
                      deadline_s: float = -1.0, stream_ptr=None) -> dict:
        """pm_measure_until: like measure, with a host deadline (seconds
        from the call, < 0: none).  Returns {"status", "t_min", "t_reps",
        "below_floor"}; status is 0 or PM_ETIMEDOUT (-6), other errors
        raise."""
        v = variant_struct(d)
        ptrs, sizes, n = self._bufs(tensors)
        tr = (ctypes.c_double * reps)()
        tmin = ctypes.c_double()
        done = ctypes.c_int32()
        flags = ctypes.c_uint32()
        rc = lib().pm_measure_until(self._h, ctypes.byref(v), ptrs, sizes, n,
                                    self._stream(stream_ptr), warmup, reps,
                                    float(deadline_s), tr, ctypes.byref(tmin),
                                    ctypes.byref(done), ctypes.byref(flags))
        if rc not in (0, -6):
            _check(rc)
        return {"status": rc, "t_min": tmin.value, "t_reps": list(tr[:done.value]),
                "below_floor": bool(flags.value & 1)}


def device_buffers(d: dict, seed: int, device: str = "cuda:0",
                   fast: bool = False):
    """Allocate the variant's buffers with torch on `device`; inputs get
    seeded uniform[-1, 1] values (synth.uniform), outputs zeros, sentinel
    outputs NaN.  Returns (tensors, host copies of the initial contents).
    fast=True draws the inputs on the device instead (same distribution,
    torch's generator; no host copies) for timing runs."""
    import torch
    if fast:
        g = torch.Generator(device=device)
        g.manual_seed(seed)
        tdt = torch.float64 if d.get("dtype", "f32") == "f64" else torch.float32
        esz = 8 if tdt == torch.float64 else 4
        out_t = []
        for nbytes, role in buffers(d):
            t = torch.empty(nbytes // esz, dtype=tdt, device=device)
            if role in (0, 2):
                t.uniform_(-1.0, 1.0, generator=g)
            elif role == 3:
                t.fill_(float("nan"))
            else:
                t.zero_()
            out_t.append(t)
        return out_t, None

    from synth import uniform
    dt = d.get("dtype", "f32")
    npdt = np.float64 if dt == "f64" else np.float32
    esz = 8 if dt == "f64" else 4
    out_t, host = [], []
    for i, (nbytes, role) in enumerate(buffers(d)):
        n = nbytes // esz
        if role in (0, 2):
            h = uniform(seed + 7919 * i, n, dt)
        elif role == 3:
            h = np.full(n, np.nan, dtype=npdt)
        else:
            h = np.zeros(n, dtype=npdt)
        host.append(h)
        out_t.append(torch.from_numpy(h).to(device))
    return out_t, host
