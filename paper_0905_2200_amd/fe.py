"""Thin ctypes binding of libfe.so (the C ABI in include/fe.h).

Argument marshalling only: tensors go in as device pointers, work is
enqueued on the context's stream (fenced against the caller's current torch
stream), every step runs in the library's HIP kernels.  There is no fallback: if the library or a GPU is
missing, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfe.so")

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EDEVICE, FE_EUNSORTED, FE_ERANGE, FE_EBUSY, FE_EINTERNAL = range(8)
FE_EXACT, FE_RELAXED = 0, 1
PARAM_SEGMENTS, PARAM_TARGET_WAVES, PARAM_MIN_SEG_EVENTS, PARAM_CONCAT_TREE, PARAM_TIMING, \
    PARAM_TYPE_DISPATCH, PARAM_CROSSOVER_A, PARAM_CROSSOVER_B, PARAM_ELIMINATION, \
    PARAM_HOST_TILING, PARAM_KEEP_CANDIDATES, PARAM_CROSSOVER_A_RELAXED, \
    PARAM_CROSSOVER_B_RELAXED, PARAM_PASS1_COST, PARAM_SAMPLE_MIN, PARAM_SHARED_LISTS = range(16)

STATUS_NAMES = {0: "FE_OK", 1: "FE_EINVAL", 2: "FE_ENOMEM", 3: "FE_EDEVICE",
                4: "FE_EUNSORTED", 5: "FE_ERANGE", 6: "FE_EBUSY", 7: "FE_EINTERNAL"}

EXPORTS = ["fe_create", "fe_destroy", "fe_last_error", "fe_sync", "fe_set_param",
           "fe_get_param", "fe_validate", "fe_count", "fe_count_noalloc", "fe_count_resume",
           "fe_count_two_pass",
           "fe_mine",
           "fe_result_free", "fe_get_stats", "fe_get_kernel_stats", "fe_reset_kernel_stats",
           "fe_batch_create", "fe_batch_run", "fe_batch_autotune", "fe_batch_set_tuning",
           "fe_batch_get_tuning", "fe_batch_destroy", "fe_count_batched",
           "fe_server_create", "fe_server_append", "fe_server_submit", "fe_server_poll",
           "fe_server_wait", "fe_server_release", "fe_server_get_stats", "fe_server_destroy"]


class FeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), msg))
        self.code = code


class _Level(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("n_candidates", ctypes.c_int64),
                ("n_survivors", ctypes.c_int64), ("n_frequent", ctypes.c_int64),
                ("types", ctypes.POINTER(ctypes.c_int32)), ("lo", ctypes.POINTER(ctypes.c_int32)),
                ("hi", ctypes.POINTER(ctypes.c_int32)), ("upper", ctypes.POINTER(ctypes.c_int32)),
                ("exact", ctypes.POINTER(ctypes.c_int32)), ("gen_ms", ctypes.c_double),
                ("count_ms", ctypes.c_double), ("passes", ctypes.c_int32),
                ("sample_n", ctypes.c_int64), ("sample_kept", ctypes.c_int64),
                ("all_types", ctypes.POINTER(ctypes.c_int32)),
                ("all_lo", ctypes.POINTER(ctypes.c_int32)),
                ("all_hi", ctypes.POINTER(ctypes.c_int32)),
                ("all_upper", ctypes.POINTER(ctypes.c_int32)),
                ("all_exact", ctypes.POINTER(ctypes.c_int32))]


class _Result(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("levels", ctypes.POINTER(_Level))]


class _Stats(ctypes.Structure):
    _fields_ = [("map_launches", ctypes.c_int64), ("segments_max", ctypes.c_int64),
                ("fallback_cands", ctypes.c_int64), ("last_call_ms", ctypes.c_double)]


class _KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("ee", ctypes.c_double)]


class _Job(ctypes.Structure):
    _fields_ = [("ids", ctypes.c_void_p), ("ticks", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("num_types", ctypes.c_int32), ("types", ctypes.c_void_p),
                ("len", ctypes.c_void_p), ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p),
                ("M", ctypes.c_int32), ("nmax", ctypes.c_int32), ("theta", ctypes.c_int32),
                ("upper_out", ctypes.c_void_p), ("exact_out", ctypes.c_void_p)]


class _Tuning(ctypes.Structure):
    _fields_ = [("seg_events", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("run_ms", ctypes.c_double)]


class _ServerCfg(ctypes.Structure):
    _fields_ = [("n_arrays", ctypes.c_int32), ("capacity", ctypes.c_int64),
                ("hbm_budget", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_round", ctypes.c_int32), ("seg_events", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("array", ctypes.c_int32), ("t_begin", ctypes.c_int32), ("t_end", ctypes.c_int32),
                ("theta", ctypes.c_int32), ("arrival_ns", ctypes.c_int64)]


class _Response(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_events", ctypes.c_int32),
                ("n_survivors", ctypes.c_int32), ("n_frequent", ctypes.c_int32),
                ("upper", ctypes.POINTER(ctypes.c_int32)), ("exact", ctypes.POINTER(ctypes.c_int32)),
                ("arrival_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("round", ctypes.c_int32),
                ("round_size", ctypes.c_int32), ("footprint", ctypes.c_int64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("largest_round", ctypes.c_int32), ("max_inflight_seen", ctypes.c_int32),
                ("budget_closed", ctypes.c_int64)]


_lib = None


def lib():
    """Load libfe.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError("libfe.so is not built: run python -m paper_0905_2200_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    V, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    CTX = ctypes.c_void_p
    sig = {
        "fe_create": ([ctypes.c_int, V, ctypes.POINTER(CTX)], ctypes.c_int),
        "fe_destroy": ([CTX], ctypes.c_int),
        "fe_last_error": ([CTX], ctypes.c_char_p),
        "fe_sync": ([CTX], ctypes.c_int),
        "fe_set_param": ([CTX, ctypes.c_int, I64], ctypes.c_int),
        "fe_get_param": ([CTX, ctypes.c_int, ctypes.POINTER(I64)], ctypes.c_int),
        "fe_validate": ([CTX, V, V, I64, I32], ctypes.c_int),
        "fe_count": ([CTX, V, V, I64, I32, V, V, V, V, I32, I32, ctypes.c_int, V], ctypes.c_int),
        "fe_count_noalloc": ([CTX, V, V, I64, I32, V, V, V, V, I32, I32, ctypes.c_int, V],
                             ctypes.c_int),
        "fe_count_two_pass": ([CTX, V, V, I64, I32, V, V, V, V, I32, I32, I32, V, V, V],
                              ctypes.c_int),
        "fe_count_resume": ([CTX, V, V, I64, I32, V, V, V, V, I32, I32, ctypes.c_int, I64, V, V],
                            ctypes.c_int),
        "fe_mine": ([CTX, V, V, I64, I32, V, V, I32, I32, I32, ctypes.POINTER(ctypes.POINTER(_Result))],
                    ctypes.c_int),
        "fe_result_free": ([ctypes.POINTER(_Result)], None),
        "fe_get_stats": ([CTX, ctypes.POINTER(_Stats)], ctypes.c_int),
        "fe_get_kernel_stats": ([CTX, ctypes.POINTER(_KStat), I32, ctypes.POINTER(I32)],
                                ctypes.c_int),
        "fe_reset_kernel_stats": ([CTX], ctypes.c_int),
        "fe_batch_create": ([CTX, I32, ctypes.POINTER(_Job), ctypes.POINTER(V)], ctypes.c_int),
        "fe_batch_run": ([V], ctypes.c_int),
        "fe_batch_autotune": ([V, I32, ctypes.POINTER(_Tuning)], ctypes.c_int),
        "fe_batch_set_tuning": ([V, ctypes.POINTER(_Tuning)], ctypes.c_int),
        "fe_batch_get_tuning": ([V, ctypes.POINTER(_Tuning)], ctypes.c_int),
        "fe_batch_destroy": ([V], ctypes.c_int),
        "fe_count_batched": ([CTX, I32, ctypes.POINTER(_Job)], ctypes.c_int),
        "fe_server_create": ([CTX, ctypes.POINTER(_ServerCfg), V, V, V, V, V, I32, I32,
                              ctypes.POINTER(V)], ctypes.c_int),
        "fe_server_append": ([V, I32, V, V, I64], ctypes.c_int),
        "fe_server_submit": ([V, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)],
                             ctypes.c_int),
        "fe_server_poll": ([V, ctypes.c_uint64, ctypes.POINTER(_Response)], ctypes.c_int),
        "fe_server_wait": ([V, ctypes.c_uint64, ctypes.POINTER(_Response)], ctypes.c_int),
        "fe_server_release": ([V, ctypes.c_uint64], ctypes.c_int),
        "fe_server_get_stats": ([V, ctypes.POINTER(_ServerStats)], ctypes.c_int),
        "fe_server_destroy": ([V], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev_i32(x, device):
    import torch
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.int32)
    else:
        t = torch.as_tensor(np.ascontiguousarray(np.asarray(x, dtype=np.int32)), device=device)
    return t.contiguous()


class Context:
    """A library context bound to one device and one torch stream.

    By default the context owns a torch stream of its own (default
    priority).  Every call first makes that stream wait for the caller's
    current stream and afterwards makes the current stream wait for it, so
    tensors produced or consumed around a call are ordered like any torch
    op on the current stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if stream is None:
            stream = torch.cuda.Stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib().fe_create(self.device.index or 0, ctypes.c_void_p(stream.cuda_stream),
                             ctypes.byref(h))
        if rc != FE_OK:
            raise FeError(rc, "fe_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().fe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ helpers
    def _enter(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _leave(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    def _call(self, fn, *args):
        self._enter()
        try:
            return fn(*args)
        finally:
            self._leave()

    def _check(self, rc):
        if rc != FE_OK:
            raise FeError(rc, lib().fe_last_error(self.h).decode())

    def set_param(self, param, value):
        self._check(lib().fe_set_param(self.h, int(param), int(value)))

    def get_param(self, param):
        v = ctypes.c_int64()
        self._check(lib().fe_get_param(self.h, int(param), ctypes.byref(v)))
        return v.value

    def stats(self):
        s = _Stats()
        self._check(lib().fe_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def kernel_stats(self):
        """{kernel kind: {launches, total_ms, max_ms, ee}} from the HIP-event
        timers (enable with set_param(PARAM_TIMING, 1))."""
        n = ctypes.c_int32()
        self._check(self._call(lib().fe_get_kernel_stats, self.h, None, 0, ctypes.byref(n)))
        arr = (_KStat * max(n.value, 1))()
        self._check(self._call(lib().fe_get_kernel_stats, self.h, arr, n.value, ctypes.byref(n)))
        return {a.name.decode(): {"launches": a.launches, "total_ms": a.total_ms,
                                  "max_ms": a.max_ms, "ee": a.ee} for a in arr[:n.value]}

    def reset_kernel_stats(self):
        self._check(self._call(lib().fe_reset_kernel_stats, self.h))

    def sync(self):
        self._check(self._call(lib().fe_sync, self.h))

    def stream_tensors(self, ids, ticks):
        return _dev_i32(ids, self.device), _dev_i32(ticks, self.device)

    def cand_tensors(self, cand):
        """Device tensors of a candidate table dict (types, len, lo, hi)."""
        d = self.device
        T = _dev_i32(cand["types"], d)
        nmax = T.shape[1] if T.dim() == 2 else 1
        M = T.shape[0]
        Ln = _dev_i32(cand["len"], d)
        lo = _dev_i32(cand["lo"], d).reshape(M, max(nmax - 1, 0)).contiguous()
        hi = _dev_i32(cand["hi"], d).reshape(M, max(nmax - 1, 0)).contiguous()
        if nmax == 1:  # keep a valid pointer for empty hop tables
            lo = self.torch.zeros((max(M, 1), 1), dtype=self.torch.int32, device=d)
            hi = lo
        return {"types": T.reshape(M, nmax), "len": Ln, "lo": lo, "hi": hi, "nmax": nmax, "M": M}

    # ------------------------------------------------------------------ API
    def validate(self, ids, ticks, num_types):
        self._check(self._call(lib().fe_validate, self.h, _ptr(ids), _ptr(ticks), ids.numel(),
                               int(num_types)))

    def count(self, ids, ticks, num_types, cand, mode=FE_EXACT, out=None):
        c = cand if "nmax" in cand and hasattr(cand["types"], "data_ptr") else self.cand_tensors(cand)
        M = c["M"]
        if out is None:
            out = self.torch.empty(max(M, 1), dtype=self.torch.int32, device=self.device)
        rc = self._call(lib().fe_count, self.h, _ptr(ids), _ptr(ticks), ids.numel(), int(num_types),
                            _ptr(c["types"]), _ptr(c["len"]), _ptr(c["lo"]), _ptr(c["hi"]),
                            M, c["nmax"], int(mode), _ptr(out))
        self._check(rc)
        return out[:M]

    def count_noalloc(self, ids, ticks, num_types, cand, mode, out):
        """fe_count_noalloc: fe_count whose workspace is the library's fixed
        device scratch (no device allocation in the call); `out` is a
        caller-allocated device int32 tensor of at least M entries."""
        c = cand if "nmax" in cand and hasattr(cand["types"], "data_ptr") else self.cand_tensors(cand)
        M = c["M"]
        rc = self._call(lib().fe_count_noalloc, self.h, _ptr(ids), _ptr(ticks), ids.numel(),
                        int(num_types), _ptr(c["types"]), _ptr(c["len"]), _ptr(c["lo"]),
                        _ptr(c["hi"]), M, c["nmax"], int(mode), _ptr(out))
        self._check(rc)
        return out[:M]

    def count_resume(self, ids, ticks, num_types, cand, mode, start, count_io, last_io):
        """Incremental count (fe_count_resume): ids/ticks hold the stream so far,
        events before `start` were counted by earlier calls; count_io / last_io
        (device int32[M]) carry counts and last completion indices and are
        updated in place."""
        c = cand if "nmax" in cand and hasattr(cand["types"], "data_ptr") else self.cand_tensors(cand)
        rc = self._call(lib().fe_count_resume, self.h, _ptr(ids), _ptr(ticks), ids.numel(),
                        int(num_types), _ptr(c["types"]), _ptr(c["len"]), _ptr(c["lo"]),
                        _ptr(c["hi"]), c["M"], c["nmax"], int(mode), int(start), _ptr(count_io),
                        _ptr(last_io))
        self._check(rc)
        return count_io, last_io

    def count_two_pass(self, ids, ticks, num_types, cand, theta, upper=None, exact=None,
                       nsurv=None):
        c = cand if "nmax" in cand and hasattr(cand["types"], "data_ptr") else self.cand_tensors(cand)
        M = c["M"]
        t = self.torch
        if upper is None:
            upper = t.empty(max(M, 1), dtype=t.int32, device=self.device)
        if exact is None:
            exact = t.empty(max(M, 1), dtype=t.int32, device=self.device)
        if nsurv is None:
            nsurv = t.zeros(1, dtype=t.int32, device=self.device)
        rc = self._call(lib().fe_count_two_pass, self.h, _ptr(ids), _ptr(ticks), ids.numel(), int(num_types),
                                     _ptr(c["types"]), _ptr(c["len"]), _ptr(c["lo"]), _ptr(c["hi"]),
                                     M, c["nmax"], int(theta), _ptr(upper), _ptr(exact),
                                     _ptr(nsurv))
        self._check(rc)
        return upper[:M], exact[:M], nsurv

    def mine(self, ids, ticks, num_types, intervals, theta, max_level):
        """Problem 1 by level-wise mining.  Returns a list of per-level dicts
        with numpy arrays (types [F, level], lo/hi [F, level-1], upper,
        exact) and the level's candidate / survivor / frequent counts."""
        ilo = np.ascontiguousarray(np.asarray([a for a, _ in intervals], np.int32))
        ihi = np.ascontiguousarray(np.asarray([b for _, b in intervals], np.int32))
        res = ctypes.POINTER(_Result)()
        rc = self._call(lib().fe_mine, self.h, _ptr(ids), _ptr(ticks), ids.numel(), int(num_types),
                           ilo.ctypes.data_as(ctypes.c_void_p), ihi.ctypes.data_as(ctypes.c_void_p),
                           len(intervals), int(theta), int(max_level), ctypes.byref(res))
        self._check(rc)
        out = []
        try:
            for i in range(res.contents.n_levels):
                L = res.contents.levels[i]
                F, lev = int(L.n_frequent), int(L.level)

                def arr(p, cnt):
                    if cnt == 0:
                        return np.zeros(0, np.int32)
                    return np.ctypeslib.as_array(p, shape=(cnt,)).copy()

                d = {
                    "level": lev, "n_candidates": int(L.n_candidates),
                    "n_survivors": int(L.n_survivors), "n_frequent": F,
                    "types": arr(L.types, F * lev).reshape(F, lev),
                    "lo": arr(L.lo, F * (lev - 1)).reshape(F, lev - 1),
                    "hi": arr(L.hi, F * (lev - 1)).reshape(F, lev - 1),
                    "upper": arr(L.upper, F), "exact": arr(L.exact, F),
                    "gen_ms": float(L.gen_ms), "count_ms": float(L.count_ms),
                    "passes": int(L.passes), "sample_n": int(L.sample_n),
                    "sample_kept": int(L.sample_kept)}
                if L.all_exact:
                    Mc = int(L.n_candidates)
                    d.update({"all_types": arr(L.all_types, Mc * lev).reshape(Mc, lev),
                              "all_lo": arr(L.all_lo, Mc * (lev - 1)).reshape(Mc, lev - 1),
                              "all_hi": arr(L.all_hi, Mc * (lev - 1)).reshape(Mc, lev - 1),
                              "all_upper": arr(L.all_upper, Mc),
                              "all_exact": arr(L.all_exact, Mc)})
                out.append(d)
        finally:
            lib().fe_result_free(res)
        return out


class Batch:
    """Two-pass counting of many recordings as one planned batch (one
    captured graph per episode size, persistent launches).  `recs` is a list
    of dicts with device tensors: ids, ticks, num_types, cand (from
    Context.cand_tensors), theta.  Outputs: self.upper[r], self.exact[r]."""

    def __init__(self, ctx, recs):
        import torch
        self.ctx = ctx
        self.recs = recs
        self.upper, self.exact = [], []
        jobs = (_Job * max(len(recs), 1))()
        for r, rec in enumerate(recs):
            c = rec["cand"]
            up = torch.empty(max(c["M"], 1), dtype=torch.int32, device=ctx.device)
            ex = torch.empty(max(c["M"], 1), dtype=torch.int32, device=ctx.device)
            self.upper.append(up[:c["M"]])
            self.exact.append(ex[:c["M"]])
            jobs[r] = _Job(rec["ids"].data_ptr(), rec["ticks"].data_ptr(), rec["ids"].numel(),
                           int(rec["num_types"]), c["types"].data_ptr(), c["len"].data_ptr(),
                           c["lo"].data_ptr(), c["hi"].data_ptr(), c["M"], c["nmax"],
                           int(rec["theta"]), up.data_ptr(), ex.data_ptr())
        self._jobs = jobs
        h = ctypes.c_void_p()
        ctx._check(ctx._call(lib().fe_batch_create, ctx.h, len(recs), jobs, ctypes.byref(h)))
        self.h = h

    def run(self):
        self.ctx._check(self.ctx._call(lib().fe_batch_run, self.h))

    def autotune(self, reps=2):
        t = _Tuning()
        self.ctx._check(self.ctx._call(lib().fe_batch_autotune, self.h, int(reps), ctypes.byref(t)))
        return {"seg_events": t.seg_events, "waves_per_cu": t.waves_per_cu,
                "waves_per_block": t.waves_per_block, "run_ms": t.run_ms}

    def set_tuning(self, seg_events, waves_per_cu, waves_per_block=0):
        t = _Tuning(int(seg_events), int(waves_per_cu), int(waves_per_block), 0.0)
        self.ctx._check(self.ctx._call(lib().fe_batch_set_tuning, self.h, ctypes.byref(t)))

    def tuning(self):
        t = _Tuning()
        self.ctx._check(lib().fe_batch_get_tuning(self.h, ctypes.byref(t)))
        return {"seg_events": t.seg_events, "waves_per_cu": t.waves_per_cu,
                "waves_per_block": t.waves_per_block, "run_ms": t.run_ms}

    def close(self):
        if getattr(self, "h", None):
            lib().fe_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Window-counting service (continuous batching of requests into rounds
    admitted by device-memory footprint, several rounds in flight).  The
    resident candidate set is a host dict (synth.pack layout); events are
    appended per array from host arrays; results come back as numpy."""

    def __init__(self, ctx, cand, num_types, capacity, hbm_budget, max_inflight=3, max_round=64,
                 seg_events=0, waves_per_cu=0):
        self.ctx = ctx
        c = ctx.cand_tensors(cand)
        self._cand = c
        self.M = c["M"]
        nt = np.ascontiguousarray(np.asarray(num_types, np.int32))
        cfg = _ServerCfg(len(nt), int(capacity), int(hbm_budget), int(max_inflight),
                         int(max_round), int(seg_events), int(waves_per_cu))
        h = ctypes.c_void_p()
        ctx.torch.cuda.synchronize(ctx.device)
        ctx._check(lib().fe_server_create(ctx.h, ctypes.byref(cfg),
                                          nt.ctypes.data_as(ctypes.c_void_p),
                                          _ptr(c["types"]), _ptr(c["len"]), _ptr(c["lo"]),
                                          _ptr(c["hi"]), self.M, c["nmax"], ctypes.byref(h)))
        self.h = h

    def append(self, array, ids, ticks):
        ids = np.ascontiguousarray(np.asarray(ids, np.int32))
        ticks = np.ascontiguousarray(np.asarray(ticks, np.int32))
        self.ctx._check(lib().fe_server_append(self.h, int(array),
                                               ids.ctypes.data_as(ctypes.c_void_p),
                                               ticks.ctypes.data_as(ctypes.c_void_p), ids.size))

    def submit(self, array, t_begin, t_end, theta, arrival_ns=0):
        r = _Request(int(array), int(t_begin), int(t_end), int(theta), int(arrival_ns))
        t = ctypes.c_uint64()
        self.ctx._check(lib().fe_server_submit(self.h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def _resp(self, r, copy):
        d = {k: getattr(r, k) for k, _ in _Response._fields_ if k not in ("upper", "exact")}
        if copy and r.upper:
            d["upper"] = np.ctypeslib.as_array(r.upper, shape=(self.M,)).copy()
            d["exact"] = np.ctypeslib.as_array(r.exact, shape=(self.M,)).copy()
        return d

    def poll(self, ticket, copy=True):
        r = _Response()
        rc = lib().fe_server_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(r))
        if rc == FE_EBUSY:
            return None
        self.ctx._check(rc)
        return self._resp(r, copy)

    def wait(self, ticket, copy=True):
        r = _Response()
        self.ctx._check(lib().fe_server_wait(self.h, ctypes.c_uint64(ticket), ctypes.byref(r)))
        return self._resp(r, copy)

    def release(self, ticket):
        self.ctx._check(lib().fe_server_release(self.h, ctypes.c_uint64(ticket)))

    def stats(self):
        s = _ServerStats()
        self.ctx._check(lib().fe_server_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().fe_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
