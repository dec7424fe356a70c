"""Python binding of libbfly.so (argument marshalling only).

Every function here forwards to the C entry point of the same name (``bf_<name>`` in
include/bfly.h).  PyTorch provides device memory and the current stream; all arithmetic
runs in the library's HIP kernels.  A missing or unloadable library raises at import of
the first call -- there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfly.so")

BF_OK, BF_EINVAL, BF_ENOMEM, BF_EBUDGET, BF_EAGAIN, BF_ENOTFOUND, BF_EHIP, BF_ECANCELED = (
    0, -1, -2, -3, -4, -5, -6, -7)
PRECISIONS = {"fp32": 0, "bf16x3": 1, "fp8": 2, "f16x2": 3, "fft": 4, "f16f8": 5, "f16f6": 6}
NORMS = {"centred": 0, "raw": 1}
STATUS_NAMES = {0: "BF_OK", -1: "BF_EINVAL", -2: "BF_ENOMEM", -3: "BF_EBUDGET",
                -4: "BF_EAGAIN", -5: "BF_ENOTFOUND", -6: "BF_EHIP", -7: "BF_ECANCELED"}
EXPORTED = ["bf_bank_bytes", "bf_bank_create", "bf_bank_info", "bf_bank_destroy",
            "bf_workspace_bytes", "bf_search_segment", "bf_search_batch", "bf_plan",
            "bf_set_timing", "bf_kernel_times", "bf_last_error",
            "bf_server_create", "bf_server_request_bytes", "bf_submit", "bf_poll", "bf_fetch",
            "bf_cancel", "bf_server_stats", "bf_server_destroy",
            "bf_tails_workspace_bytes", "bf_search_tails",
            "bf_coincidence_workspace_bytes", "bf_coincidence", "bf_search_segment_noalloc"]
STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


class BflyError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class BankDesc(ctypes.Structure):
    _fields_ = [("fs", ctypes.c_double), ("L", ctypes.c_int32), ("n_f0", ctypes.c_int32),
                ("n_fdot", ctypes.c_int32), ("shard_index", ctypes.c_int32),
                ("shard_count", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("f0_min", ctypes.c_double), ("f0_max", ctypes.c_double),
                ("fdot_min", ctypes.c_double), ("fdot_max", ctypes.c_double)]


class SearchParams(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_int32), ("t_block", ctypes.c_int32),
                ("hist_bins", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("hist_lo", ctypes.c_double), ("hist_hi", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("max_abs", ctypes.c_void_p), ("argmax", ctypes.c_void_p),
                ("spec", ctypes.c_void_p), ("spectrum", ctypes.c_void_p),
                ("hist", ctypes.c_void_p), ("n_degenerate", ctypes.c_void_p)]


class Segment(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("n", ctypes.c_int64), ("out", Result)]


class Tails(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_void_p), ("tau", ctypes.c_void_p), ("k", ctypes.c_void_p),
                ("rho", ctypes.c_void_p), ("bin_counts", ctypes.c_void_p),
                ("n_tails", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class TailSegment(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("n", ctypes.c_int64), ("out", Result),
                ("tails", Tails)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("ticks_in_flight", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("reserved2", ctypes.c_int32), ("params", SearchParams)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1802_01685_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, dp = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                            ctypes.c_void_p)
    sig = {
        "bf_bank_bytes": [ctypes.POINTER(BankDesc), ctypes.POINTER(sz)],
        "bf_bank_create": [ctypes.POINTER(BankDesc), vp, sz, vp, ctypes.POINTER(vp)],
        "bf_bank_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64), dp, dp],
        "bf_bank_destroy": [vp],
        "bf_workspace_bytes": [vp, ctypes.POINTER(i64), i32, ctypes.POINTER(SearchParams),
                               ctypes.POINTER(sz)],
        "bf_search_segment": [vp, vp, i64, ctypes.POINTER(SearchParams), ctypes.POINTER(Result),
                              vp, sz, vp],
        "bf_search_batch": [vp, ctypes.POINTER(Segment), i32, ctypes.POINTER(SearchParams), vp,
                            sz, vp],
        "bf_search_segment_noalloc": [vp, vp, i64, ctypes.POINTER(SearchParams),
                                      ctypes.POINTER(Result), vp],
        "bf_plan": [vp, ctypes.POINTER(i64), i32, ctypes.POINTER(i32), ctypes.POINTER(i64)],
        "bf_set_timing": [i32],
        "bf_kernel_times": [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)],
        "bf_server_create": [vp, ctypes.POINTER(ServerDesc), ctypes.POINTER(vp)],
        "bf_server_request_bytes": [vp, i64, ctypes.POINTER(sz)],
        "bf_submit": [vp, vp, i64, ctypes.POINTER(ctypes.c_uint64)],
        "bf_poll": [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
        "bf_fetch": [vp, ctypes.c_uint64, vp, vp, vp, vp, vp, vp],
        "bf_cancel": [vp, ctypes.c_uint64],
        "bf_server_stats": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32),
                            ctypes.POINTER(i32)],
        "bf_server_destroy": [vp],
        "bf_tails_workspace_bytes": [vp, ctypes.POINTER(i64), i32, ctypes.POINTER(SearchParams),
                                     ctypes.POINTER(sz)],
        "bf_search_tails": [vp, ctypes.POINTER(TailSegment), i32, ctypes.c_float,
                            ctypes.POINTER(SearchParams), vp, sz, vp],
        "bf_coincidence_workspace_bytes": [vp, i64, i64, ctypes.POINTER(sz)],
        "bf_coincidence": [vp, ctypes.POINTER(Tails), ctypes.POINTER(Tails), i64, i32,
                           ctypes.c_double, vp, vp, vp, vp, sz, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.bf_last_error.argtypes = []
    L.bf_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def last_error() -> str:
    return lib().bf_last_error().decode()


def _check(status: int) -> None:
    if status != BF_OK:
        raise BflyError(status, last_error())


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _record_on(stream, tensors) -> None:
    """When the work runs on a stream other than torch's current one, tell the caching
    allocator that the tensors this binding allocated are in use on that stream: otherwise a
    tensor dropped at return could be handed to the next allocation on the current stream
    while the kernels still read or write it."""
    if stream is None:
        return
    ts = stream if isinstance(stream, torch.cuda.Stream) else \
        torch.cuda.ExternalStream(_stream(stream))
    if ts.cuda_stream == torch.cuda.current_stream().cuda_stream:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(ts)


def make_desc(p, precision: str = "fp32") -> BankDesc:
    """A bank descriptor from any object with the grid attributes (fs, L, n_f0, n_fdot,
    f0_min, f0_max, fdot_min, fdot_max and optionally shard_index, shard_count)."""
    g = (lambda k, d=None: p.get(k, d)) if isinstance(p, dict) else \
        (lambda k, d=None: getattr(p, k, d))
    return BankDesc(fs=float(g("fs")), L=int(g("L")), n_f0=int(g("n_f0")),
                    n_fdot=int(g("n_fdot")), shard_index=int(g("shard_index", 0)),
                    shard_count=int(g("shard_count", 1)),
                    precision=PRECISIONS[precision] if isinstance(precision, str) else precision,
                    f0_min=float(g("f0_min")), f0_max=float(g("f0_max")),
                    fdot_min=float(g("fdot_min")), fdot_max=float(g("fdot_max")))


def make_params(norm: str = "centred", t_block: int = 1, hist_bins: int = 256,
                hist_lo: float = 0.0, hist_hi: float = 1.0) -> SearchParams:
    return SearchParams(norm=NORMS[norm] if isinstance(norm, str) else norm, t_block=t_block,
                        hist_bins=hist_bins, reserved=0, hist_lo=hist_lo, hist_hi=hist_hi)


def bank_bytes(desc: BankDesc) -> int:
    out = ctypes.c_size_t()
    _check(lib().bf_bank_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


@dataclass
class Bank:
    """A bank handle plus the torch buffer that holds its device memory."""
    handle: int
    memory: torch.Tensor
    desc: BankDesc
    K: int
    n_bins: int
    k_offset: int

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.bf_bank_destroy(ctypes.c_void_p(self.handle))
            self.handle = None

    def grid(self):
        """(f0[K], fdot[K]) of the bank's templates, float64 numpy arrays."""
        import numpy as np
        f0 = np.empty(self.K, dtype=np.float64)
        fd = np.empty(self.K, dtype=np.float64)
        _check(lib().bf_bank_info(ctypes.c_void_p(self.handle), None, None, None,
                                  f0.ctypes.data, fd.ctypes.data))
        return f0, fd


def bank_create(p, precision: str = "fp32", device=None, stream=None) -> Bank:
    """Allocates the bank's device memory with torch and builds the bank into it."""
    desc = make_desc(p, precision)
    nbytes = bank_bytes(desc)
    mem = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
    h = ctypes.c_void_p()
    _check(lib().bf_bank_create(ctypes.byref(desc), ctypes.c_void_p(mem.data_ptr()), nbytes,
                                ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
    K, nb, ko = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().bf_bank_info(h, ctypes.byref(K), ctypes.byref(nb), ctypes.byref(ko), None, None))
    return Bank(handle=h.value, memory=mem, desc=desc, K=K.value, n_bins=nb.value,
                k_offset=ko.value)


def workspace_bytes(bank: Bank, ns, params: SearchParams) -> int:
    arr = (ctypes.c_int64 * len(ns))(*[int(v) for v in ns])
    out = ctypes.c_size_t()
    _check(lib().bf_workspace_bytes(ctypes.c_void_p(bank.handle), arr, len(ns),
                                    ctypes.byref(params), ctypes.byref(out)))
    return out.value


def plan(bank: Bank, ns) -> tuple[int, int]:
    arr = (ctypes.c_int64 * len(ns))(*[int(v) for v in ns])
    r, items = ctypes.c_int32(), ctypes.c_int64()
    _check(lib().bf_plan(ctypes.c_void_p(bank.handle), arr, len(ns), ctypes.byref(r),
                         ctypes.byref(items)))
    return r.value, items.value


def alloc_outputs(bank: Bank, n: int, params: SearchParams, device,
                  want=("max_abs", "argmax", "spec", "spectrum", "hist", "n_degenerate")) -> dict:
    """torch tensors for the outputs of one series of n samples."""
    W = n - bank.desc.L + 1
    rows = -(-W // params.t_block)
    shapes = {"max_abs": ((W,), torch.float32), "argmax": ((W,), torch.int32),
              "spec": ((bank.n_bins, rows), torch.float32),      # bin-major
              "spectrum": ((bank.n_bins,), torch.float64),
              "hist": ((params.hist_bins,), torch.int32),  # uint32 bit pattern
              "n_degenerate": ((1,), torch.int64)}
    return {k: torch.empty(*shapes[k][0], dtype=shapes[k][1], device=device) for k in want}


def _result(o: dict) -> Result:
    return Result(max_abs=_ptr(o.get("max_abs")), argmax=_ptr(o.get("argmax")),
                  spec=_ptr(o.get("spec")), spectrum=_ptr(o.get("spectrum")),
                  hist=_ptr(o.get("hist")), n_degenerate=_ptr(o.get("n_degenerate")))


def alloc_workspace(bank: Bank, ns, params: SearchParams, device) -> torch.Tensor:
    return torch.empty(workspace_bytes(bank, ns, params), dtype=torch.uint8, device=device)


def search_segment(bank: Bank, x: torch.Tensor, params: SearchParams | None = None,
                   out: dict | None = None, workspace: torch.Tensor | None = None,
                   stream=None) -> dict:
    """Searches one float32 device series; returns the dict of output tensors."""
    params = params or make_params()
    assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
    n = x.shape[0]
    own = [] if out is not None else None
    out = out if out is not None else alloc_outputs(bank, n, params, x.device)
    if own is None:
        own = list(out.values())
    ws = workspace if workspace is not None else alloc_workspace(bank, [n], params, x.device)
    if workspace is None:
        own.append(ws)
    res = _result(out)
    _check(lib().bf_search_segment(ctypes.c_void_p(bank.handle), ctypes.c_void_p(x.data_ptr()),
                                   n, ctypes.byref(params), ctypes.byref(res),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   ctypes.c_void_p(_stream(stream))))
    _record_on(stream, own)
    return out


def search_segment_noalloc(bank: Bank, x: torch.Tensor, out: dict,
                           params: SearchParams | None = None, stream=None) -> dict:
    """bf_search_segment_noalloc: the search of search_segment with the library's own
    device scratch array as workspace (no allocation in the call).  The caller passes the
    output tensors (alloc_outputs); calls on one GPU must not overlap."""
    params = params or make_params()
    assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
    res = _result(out)
    _check(lib().bf_search_segment_noalloc(ctypes.c_void_p(bank.handle),
                                           ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                           ctypes.byref(params), ctypes.byref(res),
                                           ctypes.c_void_p(_stream(stream))))
    return out


def search_batch(bank: Bank, xs: list, params: SearchParams | None = None,
                 outs: list | None = None, workspace: torch.Tensor | None = None,
                 stream=None) -> list:
    """Searches several float32 device series in one pass; returns their output dicts."""
    params = params or make_params()
    ns = [int(x.shape[0]) for x in xs]
    for x in xs:
        assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
    own = []
    if outs is None:
        outs = [alloc_outputs(bank, n, params, x.device) for n, x in zip(ns, xs)]
        own += [t for o in outs for t in o.values()]
    ws = workspace if workspace is not None else alloc_workspace(bank, ns, params, xs[0].device)
    if workspace is None:
        own.append(ws)
    segs = (Segment * len(xs))()
    for i, (x, o) in enumerate(zip(xs, outs)):
        segs[i].x = x.data_ptr()
        segs[i].n = ns[i]
        segs[i].out = _result(o)
    _check(lib().bf_search_batch(ctypes.c_void_p(bank.handle), segs, len(xs),
                                 ctypes.byref(params), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), ctypes.c_void_p(_stream(stream))))
    _record_on(stream, own)
    return outs


def tails_workspace_bytes(bank: Bank, ns, params: SearchParams) -> int:
    arr = (ctypes.c_int64 * len(ns))(*[int(v) for v in ns])
    out = ctypes.c_size_t()
    _check(lib().bf_tails_workspace_bytes(ctypes.c_void_p(bank.handle), arr, len(ns),
                                          ctypes.byref(params), ctypes.byref(out)))
    return out.value


def alloc_tails(bank: Bank, capacity: int, device) -> dict:
    """torch tensors for the tail outputs of one series."""
    return {"sigma": torch.empty(bank.K, dtype=torch.float32,
                                 device=device),
            "tau": torch.empty(capacity, dtype=torch.int32, device=device),
            "k": torch.empty(capacity, dtype=torch.int32, device=device),
            "rho": torch.empty(capacity, dtype=torch.float32, device=device),
            "bin_counts": torch.empty(bank.n_bins, dtype=torch.int32, device=device),  # uint32
            "n_tails": torch.empty(1, dtype=torch.int64, device=device)}


def search_tails(bank: Bank, xs: list, kappa: float, capacity: int,
                 params: SearchParams | None = None, outs: list | None = None,
                 tails: list | None = None, workspace: torch.Tensor | None = None,
                 stream=None) -> tuple[list, list]:
    """The batched search plus the kappa-sigma tails of each float32 device series; returns
    (search output dicts, tail output dicts).  A series' tail lists hold min(n_tails,
    capacity) valid entries, in unspecified order."""
    params = params or make_params()
    ns = [int(x.shape[0]) for x in xs]
    for x in xs:
        assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
    own = []
    if outs is None:
        outs = [alloc_outputs(bank, n, params, x.device) for n, x in zip(ns, xs)]
        own += [t for o in outs for t in o.values()]
    if tails is None:
        tails = [alloc_tails(bank, capacity, x.device) for x in xs]
        own += [t for o in tails for t in o.values()]
    ws = workspace if workspace is not None else torch.empty(
        tails_workspace_bytes(bank, ns, params), dtype=torch.uint8, device=xs[0].device)
    if workspace is None:
        own.append(ws)
    segs = (TailSegment * len(xs))()
    for i, (x, o, t) in enumerate(zip(xs, outs, tails)):
        segs[i].x = x.data_ptr()
        segs[i].n = ns[i]
        segs[i].out = _result(o)
        segs[i].tails = Tails(sigma=_ptr(t["sigma"]), tau=_ptr(t["tau"]), k=_ptr(t["k"]),
                              rho=_ptr(t["rho"]), bin_counts=_ptr(t["bin_counts"]),
                              n_tails=_ptr(t["n_tails"]), capacity=int(t["tau"].numel()))
    _check(lib().bf_search_tails(ctypes.c_void_p(bank.handle), segs, len(xs),
                                 ctypes.c_float(kappa), ctypes.byref(params),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 ctypes.c_void_p(_stream(stream))))
    _record_on(stream, own)
    return outs, tails


def _tails_struct(t: dict) -> Tails:
    return Tails(sigma=_ptr(t.get("sigma")), tau=_ptr(t["tau"]), k=_ptr(t["k"]),
                 rho=_ptr(t.get("rho")), bin_counts=_ptr(t.get("bin_counts")),
                 n_tails=_ptr(t["n_tails"]), capacity=int(t["tau"].numel()))


def coincidence(bank: Bank, tails_a: dict, tails_b: dict, n_offsets: int, dtau: int,
                df: float, stream=None) -> dict:
    """Coincident tails of two channels (tail dicts of search_tails); returns device tensors
    counts_a, counts_b (uint32 bit patterns per f0 bin) and n_pairs."""
    dev = tails_a["n_tails"].device
    cap_b = int(tails_b["tau"].numel())
    nb = ctypes.c_size_t()
    _check(lib().bf_coincidence_workspace_bytes(ctypes.c_void_p(bank.handle), int(n_offsets),
                                                cap_b, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    out = {"counts_a": torch.empty(bank.n_bins, dtype=torch.int32, device=dev),
           "counts_b": torch.empty(bank.n_bins, dtype=torch.int32, device=dev),
           "n_pairs": torch.empty(1, dtype=torch.int64, device=dev)}
    ta, tb = _tails_struct(tails_a), _tails_struct(tails_b)
    _check(lib().bf_coincidence(ctypes.c_void_p(bank.handle), ctypes.byref(ta),
                                ctypes.byref(tb), int(n_offsets), int(dtau),
                                ctypes.c_double(df), ctypes.c_void_p(out["counts_a"].data_ptr()),
                                ctypes.c_void_p(out["counts_b"].data_ptr()),
                                ctypes.c_void_p(out["n_pairs"].data_ptr()),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.c_void_p(_stream(stream))))
    _record_on(stream, [ws] + list(out.values()))
    return out


def set_timing(enable: bool) -> None:
    _check(lib().bf_set_timing(1 if enable else 0))


def kernel_times() -> tuple[dict, int]:
    """Summed milliseconds per kernel over the calling thread's timed searches since the
    last call, and how many searches that was."""
    ms = (ctypes.c_double * 5)()
    cnt = ctypes.c_int32()
    _check(lib().bf_kernel_times(ms, ctypes.byref(cnt)))
    return dict(zip(("zero", "prefix", "norms", "main", "finalize"), list(ms))), cnt.value


# ---- serving ------------------------------------------------------------------------------
class Server:
    """A serving handle; keeps its bank alive."""

    def __init__(self, handle: int, bank: Bank, params: SearchParams):
        self.handle = handle
        self.bank = bank
        self.params = params

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.bf_server_destroy(ctypes.c_void_p(self.handle))
            self.handle = None


def server_create(bank: Bank, hbm_budget_bytes: int, max_slots: int = 16,
                  ticks_in_flight: int = 2, params: SearchParams | None = None) -> Server:
    params = params or make_params()
    d = ServerDesc(hbm_budget_bytes=int(hbm_budget_bytes), max_slots=max_slots,
                   ticks_in_flight=ticks_in_flight, reserved=0, reserved2=0, params=params)
    h = ctypes.c_void_p()
    _check(lib().bf_server_create(ctypes.c_void_p(bank.handle), ctypes.byref(d), ctypes.byref(h)))
    return Server(h.value, bank, params)


def server_request_bytes(server: Server, n: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().bf_server_request_bytes(ctypes.c_void_p(server.handle), int(n), ctypes.byref(out)))
    return out.value


def submit(server: Server, x) -> int:
    """Queues a float32 host series (numpy array); returns its ticket."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = ctypes.c_uint64()
    _check(lib().bf_submit(ctypes.c_void_p(server.handle), x.ctypes.data, x.shape[0],
                           ctypes.byref(t)))
    return t.value


def poll(server: Server, ticket: int) -> tuple[str, float, float, float]:
    st = ctypes.c_int32()
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().bf_poll(ctypes.c_void_p(server.handle), ticket, ctypes.byref(st),
                         ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return STATES[st.value], a.value, b.value, c.value


def fetch(server: Server, ticket: int, n: int) -> dict:
    """Outputs of a finished request of n samples as numpy arrays."""
    import numpy as np
    W = n - server.bank.desc.L + 1
    rows = -(-W // server.params.t_block)
    out = {"max_abs": np.empty(W, np.float32), "argmax": np.empty(W, np.int32),
           "spec": np.empty((server.bank.n_bins, rows), np.float32),
           "spectrum": np.empty(server.bank.n_bins, np.float64),
           "hist": np.empty(server.params.hist_bins, np.uint32),
           "n_degenerate": np.empty(1, np.int64)}
    _check(lib().bf_fetch(ctypes.c_void_p(server.handle), ticket, out["max_abs"].ctypes.data,
                          out["argmax"].ctypes.data, out["spec"].ctypes.data,
                          out["spectrum"].ctypes.data, out["hist"].ctypes.data,
                          out["n_degenerate"].ctypes.data))
    return out


def cancel(server: Server, ticket: int) -> None:
    _check(lib().bf_cancel(ctypes.c_void_p(server.handle), ticket))


def server_stats(server: Server) -> dict:
    d, t, q, o = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    c = ctypes.c_double()
    _check(lib().bf_server_stats(ctypes.c_void_p(server.handle), ctypes.byref(d), ctypes.byref(t),
                                 ctypes.byref(c), ctypes.byref(q), ctypes.byref(o)))
    return {"done": d.value, "ticks": t.value, "correlations": c.value, "queued": q.value,
            "on_device": o.value}


def server_destroy(server: Server) -> None:
    if server.handle:
        _check(lib().bf_server_destroy(ctypes.c_void_p(server.handle)))
        server.handle = None
