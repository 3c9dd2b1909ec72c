"""MI355X block-based triangle counting (bbTC, arXiv 2009.12457).

Thin ctypes binding over ``libbbtc.so`` (C ABI in ``include/bbtc.h``).  The
functions keep the C names; they only marshal arguments.  Every step of the
computation -- degree ordering, orientation, the symmetric rectilinear cut,
the block row index and the per-task counts -- runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.

There is no fallback: if the library is missing, importing this package
raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbtc.so")

BBTC_OK = 0
BBTC_EINVAL = -1
BBTC_ENOMEM = -2
BBTC_EBUDGET = -3
BBTC_EDEVICE = -4
BBTC_ESTATE = -5
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EBUDGET", -4: "EDEVICE", -5: "ESTATE"}

BBTC_CSR_DEVICE = 1
BBTC_CSR_TRUSTED = 2

BBTC_MODE_PERSISTENT = 0
BBTC_MODE_PLAIN_INTERSECT = 1
BBTC_MODE_PLAIN_HMAP = 2
BBTC_CUT_BALANCED = 0
BBTC_CUT_UNIFORM = 1
BBTC_TASK_EMPTY = 0
BBTC_TASK_WORK = 1


class bbtc_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("rowptr_bits", ctypes.c_int32), ("flags", ctypes.c_uint32), ("colidx", ctypes.c_void_p)]


class bbtc_options(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("cut_mode", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("wave_min", ctypes.c_int32), ("hash_min", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("item_rows", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("device_budget_bytes", ctypes.c_int64), ("bound_min_deg", ctypes.c_int32),
                ("dense", ctypes.c_int32)]


class bbtc_task(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("j", ctypes.c_int32), ("k", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("est", ctypes.c_double)]


class bbtc_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("p", ctypes.c_int64), ("ntasks", ctypes.c_int64),
                ("work_tasks", ctypes.c_int64), ("nitems", ctypes.c_int64), ("m_max", ctypes.c_int64),
                ("m_avg", ctypes.c_double), ("lambda_", ctypes.c_double), ("d_max", ctypes.c_int64),
                ("d_max_block", ctypes.c_int64), ("c", ctypes.c_double), ("wedges", ctypes.c_int64),
                ("bytes_colidx", ctypes.c_int64), ("bytes_rowidx", ctypes.c_int64),
                ("bytes_total", ctypes.c_int64), ("footprint", ctypes.c_int64), ("partition_ms", ctypes.c_double),
                ("streamed", ctypes.c_int64), ("stripe_slots", ctypes.c_int64), ("stripe_bytes", ctypes.c_int64),
                ("stripe_uploads", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("stored_rows", ctypes.c_int64), ("bound_bytes", ctypes.c_int64),
                ("dense_slices", ctypes.c_int64), ("dense_bytes", ctypes.c_int64)]


class bbtc_hybrid_stats(ctypes.Structure):
    _fields_ = [("gpu_tasks", ctypes.c_int64), ("cpu_tasks", ctypes.c_int64), ("gpu_launches", ctypes.c_int64),
                ("cutoff", ctypes.c_int64), ("split", ctypes.c_int64), ("cpu_threads", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("cpu_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("cpu_triangles", ctypes.c_uint64)]


class bbtc_tables(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("p", ctypes.c_int32), ("rT", ctypes.c_int32),
                ("cuts", ctypes.c_void_p), ("orow", ctypes.c_void_p), ("ocol", ctypes.c_void_p),
                ("botp", ctypes.c_void_p), ("bot", ctypes.c_void_p), ("acp", ctypes.c_void_p),
                ("acol", ctypes.c_void_p), ("aoff", ctypes.c_void_p), ("icolb", ctypes.c_void_p)]


TASK_DTYPE = np.dtype([("i", np.int32), ("j", np.int32), ("k", np.int32), ("kind", np.int32), ("est", np.float64)])

# Every function the header declares, with ctypes signatures.
_P = ctypes.c_void_p
_SIGS = {
    "bbtc_options_default": (None, [ctypes.POINTER(bbtc_options)]),
    "bbtc_partition": (ctypes.c_int32, [ctypes.POINTER(bbtc_csr), ctypes.POINTER(bbtc_options), _P,
                                        ctypes.POINTER(_P)]),
    "bbtc_count": (ctypes.c_int32, [_P, _P, _P, _P]),
    "bbtc_count_multi": (ctypes.c_int32, [ctypes.POINTER(_P), ctypes.c_int32, _P, ctypes.POINTER(_P), _P]),
    "bbtc_count_multi_static": (ctypes.c_int32, [ctypes.POINTER(_P), ctypes.c_int32, _P, ctypes.POINTER(_P), _P]),
    "bbtc_count_hybrid": (ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.POINTER(bbtc_hybrid_stats)]),
    "bbtc_autotune": (ctypes.c_int32, [ctypes.POINTER(bbtc_csr), ctypes.POINTER(bbtc_options), ctypes.c_int32, _P,
                                       ctypes.POINTER(bbtc_options), ctypes.POINTER(ctypes.c_double)]),
    "bbtc_plan_tasks": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.POINTER(bbtc_task)),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "bbtc_plan_cuts": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "bbtc_plan_block_nnz": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.POINTER(ctypes.c_int64)),
                                             ctypes.POINTER(ctypes.c_int64)]),
    "bbtc_plan_stats": (ctypes.c_int32, [_P, ctypes.POINTER(bbtc_stats)]),
    "bbtc_plan_copy_perm": (ctypes.c_int32, [_P, _P, _P]),
    "bbtc_plan_copy_oriented": (ctypes.c_int32, [_P, _P, _P, _P]),
    "bbtc_plan_destroy": (None, [_P]),
    "bbtc_check_tables": (ctypes.c_int32, [ctypes.POINTER(bbtc_tables)]),
    "bbtc_plan_verify": (ctypes.c_int32, [_P, _P]),
    "bbtc_last_error": (ctypes.c_char_p, []),
}


def _load():
    # torch first: libbbtc.so then binds to the HIP runtime that torch has
    # already loaded (same soname), so one runtime owns every device pointer
    # and stream in the process.  Loaded the other way round, the process
    # would hold two runtimes and the library would not recognise torch's
    # allocations.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build() or "
                          f"python paper_2009_12457_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


class BbtcError(RuntimeError):
    def __init__(self, status, where):
        self.status = int(status)
        msg = _lib.bbtc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_STATUS.get(self.status, self.status)}: {msg}")


def _check(st, where):
    if st != BBTC_OK:
        raise BbtcError(st, where)


def bbtc_last_error() -> str:
    return _lib.bbtc_last_error().decode(errors="replace")


def bbtc_options_default(**kw) -> bbtc_options:
    o = bbtc_options()
    _lib.bbtc_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, int(v))
    return o


def _stream_handle(stream):
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _array_ptr(a):
    """(pointer, on_device, itemsize, keepalive) for a numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a)
        return a.ctypes.data, False, a.dtype.itemsize, a
    import torch
    if isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            a = a.contiguous()
        return a.data_ptr(), a.is_cuda, a.element_size(), a
    raise TypeError(f"unsupported array type {type(a)}")


class Plan:
    """An opaque bbtc_plan* with borrowed views of its host-side metadata."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def _need(self):
        if not self._h.value:
            raise BbtcError(BBTC_ESTATE, "plan destroyed")

    def tasks(self) -> np.ndarray:
        self._need()
        ptr = ctypes.POINTER(bbtc_task)()
        nt = ctypes.c_int64()
        _check(_lib.bbtc_plan_tasks(self._h, ctypes.byref(ptr), ctypes.byref(nt)), "bbtc_plan_tasks")
        if nt.value == 0:
            return np.zeros(0, TASK_DTYPE)
        buf = ctypes.cast(ptr, ctypes.POINTER(ctypes.c_char * (nt.value * TASK_DTYPE.itemsize))).contents
        return np.frombuffer(bytes(buf), dtype=TASK_DTYPE).copy()

    def cuts(self) -> np.ndarray:
        self._need()
        ptr = ctypes.POINTER(ctypes.c_int32)()
        p = ctypes.c_int32()
        _check(_lib.bbtc_plan_cuts(self._h, ctypes.byref(ptr), ctypes.byref(p)), "bbtc_plan_cuts")
        return np.ctypeslib.as_array(ptr, shape=(p.value + 1,)).copy()

    def block_nnz(self) -> np.ndarray:
        self._need()
        ptr = ctypes.POINTER(ctypes.c_int64)()
        nb = ctypes.c_int64()
        _check(_lib.bbtc_plan_block_nnz(self._h, ctypes.byref(ptr), ctypes.byref(nb)), "bbtc_plan_block_nnz")
        return np.ctypeslib.as_array(ptr, shape=(nb.value,)).copy()

    def stats(self) -> dict:
        self._need()
        s = bbtc_stats()
        _check(_lib.bbtc_plan_stats(self._h, ctypes.byref(s)), "bbtc_plan_stats")
        d = {f: getattr(s, f) for f, _ in bbtc_stats._fields_}
        d["lambda"] = d.pop("lambda_")
        return d

    @property
    def ntasks(self) -> int:
        return int(self.stats()["ntasks"])

    def perm(self, stream=None) -> np.ndarray:
        """Rank of every original vertex id (synchronises the stream)."""
        import torch
        st = self.stats()
        out = torch.empty(int(st["n"]), dtype=torch.int32, device="cuda")
        _check(_lib.bbtc_plan_copy_perm(self._h, ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
               "bbtc_plan_copy_perm")
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def oriented(self, stream=None):
        """(orow uint32[n+1], ocol int32[m]) of the degree-ordered oriented CSR."""
        import torch
        st = self.stats()
        orow = torch.empty(int(st["n"]) + 1, dtype=torch.int32, device="cuda")
        ocol = torch.empty(max(int(st["m"]), 1), dtype=torch.int32, device="cuda")
        _check(_lib.bbtc_plan_copy_oriented(self._h, ctypes.c_void_p(orow.data_ptr()),
                                            ctypes.c_void_p(ocol.data_ptr()), _stream_handle(stream)),
               "bbtc_plan_copy_oriented")
        torch.cuda.synchronize()
        return orow.cpu().numpy().view(np.uint32), ocol.cpu().numpy()[:int(st["m"])]

    def verify(self, stream=None):
        """bbtc_plan_verify: the plan's tables and work items are consistent
        (raises BbtcError naming the first violation otherwise)."""
        self._need()
        _check(_lib.bbtc_plan_verify(self._h, _stream_handle(stream)), "bbtc_plan_verify")

    def destroy(self):
        if self._h.value:
            _lib.bbtc_plan_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _csr_struct(n, rowptr, colidx, trusted):
    rp, rp_dev, rp_size, keep_rp = _array_ptr(rowptr)
    ci, ci_dev, ci_size, keep_ci = _array_ptr(colidx)
    if rp_size not in (4, 8) or ci_size != 4:
        raise TypeError("rowptr must be int32/int64 and colidx int32")
    if rp_dev != ci_dev:
        raise ValueError("rowptr and colidx must both be on the host or both on the device")
    nnz = int(keep_ci.shape[0])
    g = bbtc_csr(n=int(n), nnz=nnz, rowptr=rp, rowptr_bits=8 * rp_size,
                 flags=(BBTC_CSR_DEVICE if rp_dev else 0) | (BBTC_CSR_TRUSTED if trusted else 0),
                 colidx=ci if nnz else None)
    return g, (keep_rp, keep_ci)


_TUNED = ("p", "wave_min", "hash_min")  # the fields the autotuner chooses


def _library_digest() -> str:
    """Digest of the loaded library file: cached timings are only valid for
    the kernels they were measured with."""
    import hashlib
    h = hashlib.sha256()
    with open(LIB_PATH, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:16]


def bbtc_autotune(n, rowptr, colidx, base=None, reps: int = 3, stream=None, trusted: bool = False,
                  cache_path: str | None = None):
    """Chosen options (and count ms) for this graph; optionally cached in a
    JSON file keyed by a signature of the graph (n, nnz, degree moments),
    every field of `base` and the library build.  A cache hit copies only the
    tuned fields (p, wave_min, hash_min) onto `base`."""
    import json
    key = None
    base_opts = base if base is not None else bbtc_options_default()
    if cache_path:
        rp = rowptr if isinstance(rowptr, np.ndarray) else rowptr.detach().cpu().numpy()
        deg = np.diff(rp.astype(np.int64))
        key = f"n{int(n)}-nnz{int(rp[-1])}-d2{int((deg * deg).sum())}-dmax{int(deg.max()) if len(deg) else 0}"
        key += "-" + "-".join(f"{f}{getattr(base_opts, f)}" for f, _ in bbtc_options._fields_)
        key += "-lib" + _library_digest()
        if os.path.exists(cache_path):
            cache = json.load(open(cache_path))
            if key in cache:
                rec = cache[key]
                out = bbtc_options_default(**{f: getattr(base_opts, f) for f, _ in bbtc_options._fields_})
                for f in _TUNED:
                    setattr(out, f, int(rec["options"][f]))
                return out, rec["ms"]
    g, keep = _csr_struct(n, rowptr, colidx, trusted)
    out = bbtc_options()
    ms = ctypes.c_double()
    _check(_lib.bbtc_autotune(ctypes.byref(g), ctypes.byref(base) if base is not None else None, int(reps),
                              _stream_handle(stream), ctypes.byref(out), ctypes.byref(ms)), "bbtc_autotune")
    if cache_path:
        cache = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        cache[key] = {"options": {f: getattr(out, f) for f, _ in bbtc_options._fields_}, "ms": ms.value}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return out, ms.value


def bbtc_partition(n, rowptr, colidx, options=None, stream=None, plan: Plan | None = None,
                   trusted: bool = False) -> Plan:
    """Builds (or rebuilds in place) a plan for a symmetric CSR graph.

    rowptr/colidx: numpy arrays (host) or torch tensors (host or device);
    rowptr int32 or int64, colidx int32.
    """
    g, keep = _csr_struct(n, rowptr, colidx, trusted)
    opt = options if options is not None else bbtc_options_default()
    h = ctypes.c_void_p(plan.handle.value if plan is not None else None)
    st = _lib.bbtc_partition(ctypes.byref(g), ctypes.byref(opt), _stream_handle(stream), ctypes.byref(h))
    _check(st, "bbtc_partition")
    if plan is not None:
        plan._h = h
        return plan
    return Plan(h.value)


def bbtc_count(plan: Plan, per_task=None, total=None, stream=None):
    """Enqueues the count.  Returns (per_task, total) int64 device tensors
    holding the uint64 counts (every count here is far below 2^63)."""
    import torch
    nt = plan.ntasks
    if per_task is None:
        per_task = torch.empty(max(nt, 1), dtype=torch.int64, device="cuda")
    if total is None:
        total = torch.empty(1, dtype=torch.int64, device="cuda")
    _check(_lib.bbtc_count(plan.handle, _stream_handle(stream), ctypes.c_void_p(per_task.data_ptr()),
                           ctypes.c_void_p(total.data_ptr())), "bbtc_count")
    return per_task, total


def bbtc_count_hybrid(plan: Plan, per_task=None, total=None, stream=None, cpu_threads: int = 0, cutoff: int = -1):
    """GPU and host threads count the plan together (synchronous).  Returns
    (per_task, total, stats) with per_task/total as bbtc_count's."""
    import torch
    nt = plan.ntasks
    if per_task is None:
        per_task = torch.empty(max(nt, 1), dtype=torch.int64, device="cuda")
    if total is None:
        total = torch.empty(1, dtype=torch.int64, device="cuda")
    st = bbtc_hybrid_stats()
    _check(_lib.bbtc_count_hybrid(plan.handle, _stream_handle(stream), ctypes.c_void_p(per_task.data_ptr()),
                                  ctypes.c_void_p(total.data_ptr()), int(cpu_threads), int(cutoff),
                                  ctypes.byref(st)), "bbtc_count_hybrid")
    return per_task, total, {f: getattr(st, f) for f, _ in bbtc_hybrid_stats._fields_ if f != "pad"}


BBTC_STATIC_MAX_PLANS = 64


def bbtc_count_multi(plans, per_task_list=None, totals=None, stream=None, static=False):
    """Shared persistent launch over several plans.  static=True calls
    bbtc_count_multi_static (launch state in the library's fixed device
    array, no allocation inside the call)."""
    import torch
    k = len(plans)
    if per_task_list is None:
        per_task_list = [torch.empty(max(p.ntasks, 1), dtype=torch.int64, device="cuda") for p in plans]
    if totals is None:
        totals = torch.empty(max(k, 1), dtype=torch.int64, device="cuda")
    arr = (ctypes.c_void_p * max(k, 1))(*[p.handle.value for p in plans])
    outs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in per_task_list])
    fn, name = ((_lib.bbtc_count_multi_static, "bbtc_count_multi_static") if static
                else (_lib.bbtc_count_multi, "bbtc_count_multi"))
    _check(fn(arr, k, _stream_handle(stream), outs, ctypes.c_void_p(totals.data_ptr())), name)
    return per_task_list, totals


def bbtc_check_tables(n, m, p, rT, cuts, orow, ocol, botp, bot, acp, acol, aoff, icolb):
    """bbtc_check_tables on host numpy arrays (dtypes as the header states)."""
    want = {"cuts": np.int32, "orow": np.uint32, "ocol": np.int32, "botp": np.uint64, "bot": np.uint32,
            "acp": np.uint64, "acol": np.int32, "aoff": np.uint32, "icolb": np.int32}
    loc = dict(cuts=cuts, orow=orow, ocol=ocol, botp=botp, bot=bot, acp=acp, acol=acol, aoff=aoff, icolb=icolb)
    arrs = {}
    for k, dt in want.items():
        a = np.ascontiguousarray(loc[k], dtype=dt)
        arrs[k] = a if a.size else np.zeros(1, dt)
    t = bbtc_tables(n=int(n), m=int(m), p=int(p), rT=int(rT), **{k: a.ctypes.data for k, a in arrs.items()})
    _check(_lib.bbtc_check_tables(ctypes.byref(t)), "bbtc_check_tables")


def csr_of(graph, device=None):
    """(n, rowptr, colidx) of a graphgen.Graph, optionally as device tensors."""
    if device is None:
        return graph.n, graph.rowptr, graph.colidx
    import torch
    return (graph.n, torch.from_numpy(graph.rowptr).to(device), torch.from_numpy(graph.colidx).to(device))
