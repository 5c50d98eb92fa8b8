"""Python binding of libbtprice (include/bt.h): ask and bid prices of
American options under proportional transaction costs and the zero-cost CRR
price, computed by HIP kernels on an MI355X.

The binding only marshals arguments; every step of the pricing runs in the
library's kernels.  PyTorch supplies device memory and streams.  The library
is built in-tree by ``paper_1110_2477_amd/build.py``; without it every call
raises ``RuntimeError`` -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

from .workloads import GRAD_DTYPE, HEDGE_DTYPE, PARAMS_DTYPE, RESULT_DTYPE  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbtprice.so")

BT_OK, BT_EINVAL, BT_ENOMEM, BT_EHIP, BT_EOVERFLOW, BT_ENOSUPP = 0, -1, -2, -3, -4, -5
PUT, CALL, BULL, PUT_CASH, CALL_CASH, BEAR, STRADDLE = 0, 1, 2, 3, 4, 5, 6
EUROPEAN, COST_AT_T0 = 1, 2

# Function names declared in include/bt.h.
ABI_FUNCTIONS = ("bt_autotune", "bt_book_create", "bt_book_info", "bt_book_price", "bt_book_price_grad",
                 "bt_book_price_hedge", "bt_book_price_exercise",
                 "bt_book_resolve_overflow", "bt_book_timings", "bt_book_destroy", "bt_price", "bt_shutdown",
                 "bt_price_batch", "bt_price_grad_batch", "bt_price_adjoint_batch", "bt_price_batch_static",
                 "bt_model_constants",
                 "bt_strerror",
                 "bt_version", "bt_last_hip_error")


class BtError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


BT_TUNE_TIMING = 1
BT_TUNE_GREEKS = 2
BT_TUNE_GRAPH = 4
KERNEL_NAMES = ("setup", "bid", "ask", "price0")


BT_AUTOTUNE_CANDIDATES = 6   # the library's own candidate list (include/bt.h)


class _Tune(ctypes.Structure):
    _fields_ = [("wgs_per_cu", ctypes.c_int32), ("level_factor", ctypes.c_int32),
                ("pool_points", ctypes.c_int32), ("flags", ctypes.c_int32), ("band_levels", ctypes.c_int32)]

    @classmethod
    def of(cls, tune):
        return cls(*(int(tune.get(f, 0)) for f, _ in cls._fields_))

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def lib():
    """The loaded libbtprice (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1110_2477_amd/build.py "
                           "(the HIP path has no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    L.bt_book_create.argtypes = [vp, i32, vp, ctypes.POINTER(vp)]
    L.bt_book_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), i64p]
    L.bt_book_price.argtypes = [vp, vp, vp]
    L.bt_book_price_grad.argtypes = [vp, vp, vp, vp]
    L.bt_book_price_hedge.argtypes = [vp, vp, vp, vp]
    L.bt_book_price_exercise.argtypes = [vp, vp, vp, vp]
    L.bt_book_timings.argtypes = [vp, dp, ctypes.POINTER(i32)]
    L.bt_book_resolve_overflow.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i32)]
    L.bt_book_destroy.argtypes = [vp]
    L.bt_autotune.argtypes = [vp, i32, vp, vp, i32, i32, vp, vp, dp]
    L.bt_book_destroy.restype = None
    L.bt_price.argtypes = [vp, vp]
    L.bt_price_batch.argtypes = [vp, i32, i32, vp, vp, vp]
    L.bt_price_grad_batch.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.bt_price_batch_static.argtypes = [vp, i32, i32, vp, vp]
    L.bt_price_adjoint_batch.argtypes = [vp, i32, i32, vp, vp, vp]
    L.bt_shutdown.argtypes = []
    L.bt_model_constants.argtypes = [vp, dp, dp, dp, dp, dp]
    L.bt_strerror.argtypes = [ctypes.c_int]
    L.bt_strerror.restype = ctypes.c_char_p
    L.bt_version.argtypes = []
    L.bt_last_hip_error.argtypes = []
    for f in ("bt_autotune", "bt_book_create", "bt_book_info", "bt_book_price", "bt_book_price_grad",
              "bt_book_price_hedge", "bt_book_price_exercise", "bt_book_timings", "bt_book_resolve_overflow",
              "bt_price", "bt_shutdown", "bt_model_constants", "bt_version", "bt_last_hip_error",
              "bt_price_batch", "bt_price_grad_batch", "bt_price_batch_static", "bt_price_adjoint_batch"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def strerror(code):
    return lib().bt_strerror(int(code)).decode()


def bt_version():
    return lib().bt_version()


def _check(rc, what):
    if rc != BT_OK:
        raise BtError(rc, what)


def _params(params):
    p = np.ascontiguousarray(np.asarray(params, dtype=PARAMS_DTYPE).reshape(-1))
    return p


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def bt_book_create(params, tune=None):
    """Creates a book (opaque handle) from a PARAMS_DTYPE array."""
    p = _params(params)
    h = ctypes.c_void_p()
    t = _Tune.of(tune) if tune is not None else None
    rc = lib().bt_book_create(p.ctypes.data, len(p), ctypes.byref(t) if t is not None else None,
                              ctypes.byref(h))
    _check(rc, "bt_book_create")
    return h


def bt_autotune(params, base=None, candidates=None, reps=1, stream=None):
    """Times candidate tunings of a book of `params` on the GPU and returns
    (best tune dict, [(candidate dict, ms per call), ...]); candidates=None
    takes the library's list (band_levels x wgs_per_cu)."""
    p = _params(params)
    b = _Tune.of(base) if base is not None else None
    cand = None
    n_cand = BT_AUTOTUNE_CANDIDATES
    if candidates is not None:
        cand = (_Tune * len(candidates))(*[_Tune.of(c) for c in candidates])
        n_cand = len(candidates)
    ms = (ctypes.c_double * n_cand)()
    best = _Tune()
    rc = lib().bt_autotune(p.ctypes.data, len(p), ctypes.byref(b) if b is not None else None,
                           ctypes.cast(cand, ctypes.c_void_p) if cand is not None else None,
                           n_cand if cand is not None else 0, int(reps), _stream_ptr(stream), ctypes.byref(best), ms)
    _check(rc, "bt_autotune")
    if cand is not None:
        listed = [c.as_dict() for c in cand]
    else:
        b0 = b.as_dict() if b is not None else _Tune().as_dict()
        listed = [dict(b0, band_levels=band, wgs_per_cu=w) for band in (8, 16, 32) for w in (1, 2)]
    return best.as_dict(), list(zip(listed, list(ms)))


def bt_book_info(book):
    n, nmax, nodes = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().bt_book_info(book, ctypes.byref(n), ctypes.byref(nmax), ctypes.byref(nodes)),
           "bt_book_info")
    return n.value, nmax.value, nodes.value


def bt_book_price(book, d_out_ptr, stream=None):
    """Launches the pricing of a book into device memory at ``d_out_ptr``
    (n bt_result records) on ``stream`` (a torch stream, a raw handle or None
    for torch's current stream)."""
    _check(lib().bt_book_price(book, ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(_stream_ptr(stream))),
           "bt_book_price")


def bt_book_price_grad(book, d_out_ptr, d_grad_ptr, stream=None):
    _check(lib().bt_book_price_grad(book, ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(d_grad_ptr),
                                    ctypes.c_void_p(_stream_ptr(stream))), "bt_book_price_grad")


def bt_book_resolve_overflow(book, d_out_ptr, d_grad_ptr=0, stream=None):
    """Re-prices the options of a finished call that overflowed the book's
    level buffers (with their Greeks when d_grad_ptr is the Greeks buffer of
    a bt_book_price_grad call); returns how many still overflow."""
    rem = ctypes.c_int32()
    _check(lib().bt_book_resolve_overflow(book, ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(d_grad_ptr or None),
                                          ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(rem)),
           "bt_book_resolve_overflow")
    return rem.value


def bt_book_timings(book):
    """Per-kernel milliseconds summed over the pricing calls since the last
    query (book created with flags=BT_TUNE_TIMING), and the call count."""
    ms = (ctypes.c_double * 4)()
    calls = ctypes.c_int32()
    _check(lib().bt_book_timings(book, ms, ctypes.byref(calls)), "bt_book_timings")
    return dict(zip(KERNEL_NAMES, list(ms))), calls.value


def bt_book_destroy(book):
    lib().bt_book_destroy(book)


def bt_price(params):
    """Plain single-option pricing (host in, host out, synchronous)."""
    p = _params(params)
    if len(p) != 1:
        raise ValueError("bt_price takes one option")
    out = np.zeros(1, dtype=RESULT_DTYPE)
    _check(lib().bt_price(p.ctypes.data, out.ctypes.data), "bt_price")
    return out[0]


def bt_price_batch(d_params_ptr, n, max_N, d_out_ptr, stream=None, tune=None):
    """Batch pricing of n bt_params records at device address d_params_ptr
    into n bt_result records at d_out_ptr, on ``stream`` (torch's current
    stream when None); every option's N must be at most max_N."""
    t = _Tune.of(tune) if tune is not None else None
    _check(lib().bt_price_batch(ctypes.c_void_p(d_params_ptr), int(n), int(max_N), ctypes.c_void_p(d_out_ptr),
                                ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(t) if t is not None else None),
           "bt_price_batch")


def bt_price_grad_batch(d_params_ptr, n, max_N, d_out_ptr, d_grad_ptr, stream=None, tune=None):
    """As bt_price_batch, plus n bt_grad records at d_grad_ptr."""
    t = _Tune.of(tune) if tune is not None else None
    _check(lib().bt_price_grad_batch(ctypes.c_void_p(d_params_ptr), int(n), int(max_N),
                                     ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(d_grad_ptr),
                                     ctypes.c_void_p(_stream_ptr(stream)),
                                     ctypes.byref(t) if t is not None else None), "bt_price_grad_batch")


def bt_price_adjoint_batch(d_params_ptr, n, max_N, d_out_ptr, d_grad_ptr, stream=None):
    """Prices and reverse-mode Greeks (checkpointed reverse sweep) of n
    bt_params records in device memory."""
    _check(lib().bt_price_adjoint_batch(ctypes.c_void_p(d_params_ptr), int(n), int(max_N),
                                        ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(d_grad_ptr),
                                        ctypes.c_void_p(_stream_ptr(stream))), "bt_price_adjoint_batch")


def bt_price_batch_static(d_params_ptr, n, max_N, d_out_ptr, stream=None):
    """The no-allocation variant of bt_price_batch (include/bt.h): the
    library's fixed device scratch array, at most BT_STATIC_MAX_OPTIONS
    options of at most BT_STATIC_MAX_N steps."""
    _check(lib().bt_price_batch_static(ctypes.c_void_p(d_params_ptr), int(n), int(max_N),
                                       ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(_stream_ptr(stream))),
           "bt_price_batch_static")


BT_STATIC_MAX_OPTIONS = 64
BT_STATIC_MAX_N = 1024
BT_MAX_N = 65536


def params_tensor(params, device="cuda"):
    """A uint8 device tensor holding PARAMS_DTYPE records (the layout of
    bt_params)."""
    import torch
    p = _params(params)
    return torch.from_numpy(p.view(np.uint8).copy()).to(device)


def price_batch(d_params, max_N, grad=False, stream=None, tune=None, mode="forward"):
    """Prices the bt_params records of the uint8 device tensor ``d_params``
    (see params_tensor) on the GPU; returns uint8 device tensors of bt_result
    records (and of bt_grad records with grad=True: carried tangents with
    mode="forward", the checkpointed reverse sweep with mode="adjoint").
    Asynchronous on ``stream``; nothing is copied to the host."""
    import torch
    n = d_params.numel() // PARAMS_DTYPE.itemsize
    if d_params.dtype != torch.uint8 or not d_params.is_cuda or not d_params.is_contiguous() \
            or d_params.numel() != n * PARAMS_DTYPE.itemsize:
        raise ValueError("d_params must be a contiguous uint8 CUDA tensor of bt_params records")
    out = torch.empty(n * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=d_params.device)
    if not grad:
        bt_price_batch(d_params.data_ptr(), n, max_N, out.data_ptr(), stream, tune)
        return out
    g = torch.empty(n * GRAD_DTYPE.itemsize, dtype=torch.uint8, device=d_params.device)
    if mode == "adjoint":
        bt_price_adjoint_batch(d_params.data_ptr(), n, max_N, out.data_ptr(), g.data_ptr(), stream)
    elif mode == "forward":
        bt_price_grad_batch(d_params.data_ptr(), n, max_N, out.data_ptr(), g.data_ptr(), stream, tune)
    else:
        raise ValueError(f"mode must be 'forward' or 'adjoint', not {mode!r}")
    return out, g


def as_results(t):
    """RESULT_DTYPE array of a uint8 tensor of bt_result records (copies to the host)."""
    return np.frombuffer(t.cpu().numpy().tobytes(), dtype=RESULT_DTYPE).copy()


def as_grads(t):
    """GRAD_DTYPE array of a uint8 tensor of bt_grad records (copies to the host)."""
    return np.frombuffer(t.cpu().numpy().tobytes(), dtype=GRAD_DTYPE).copy()


def bt_shutdown():
    """Frees bt_price's cached book of the calling thread and every batch
    workspace."""
    _check(lib().bt_shutdown(), "bt_shutdown")


def bt_model_constants(params):
    p = _params(params)
    vals = [ctypes.c_double() for _ in range(5)]
    rc = lib().bt_model_constants(p.ctypes.data, *[ctypes.byref(v) for v in vals])
    _check(rc, "bt_model_constants")
    return dict(zip(("u", "d", "r", "rho", "p"), (v.value for v in vals)))


CPU_LIB_PATH = os.path.join(HERE, "libbtcpu.so")
_cpu = None


class _CpuStats(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("nodes", ctypes.c_int64 * 64), ("threads", ctypes.c_int32),
                ("rounds", ctypes.c_int32)]


def cpu_lib():
    """The loaded libbtcpu (the paper's Algorithm 1 on host threads)."""
    global _cpu
    if _cpu is not None:
        return _cpu
    if not os.path.exists(CPU_LIB_PATH):
        raise RuntimeError(f"{CPU_LIB_PATH} is missing: build it with paper_1110_2477_amd/build.py")
    L = ctypes.CDLL(CPU_LIB_PATH)
    L.bt_cpu_price.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    L.bt_cpu_price.restype = ctypes.c_int
    _cpu = L
    return L


def cpu_price(params, threads, L=5):
    """One option by Algorithm 1 (Section 4.2) on `threads` host threads with
    at most L levels per round; returns (RESULT_DTYPE record, stats dict with
    seconds, per-thread node counts and rounds)."""
    p = _params(params)
    if len(p) != 1:
        raise ValueError("cpu_price takes one option")
    out = np.zeros(1, dtype=RESULT_DTYPE)
    st = _CpuStats()
    _check(cpu_lib().bt_cpu_price(p.ctypes.data, int(threads), int(L), out.ctypes.data, ctypes.byref(st)),
           "bt_cpu_price")
    return out[0], dict(seconds=st.seconds, nodes=list(st.nodes[:int(threads)]), rounds=int(st.rounds))


class Book:
    """A priced-repeatedly batch of options on the current GPU.

    ``price()`` returns a uint8 CUDA tensor holding n bt_result records;
    ``results()`` copies it to a RESULT_DTYPE numpy array.  With
    ``greeks=True`` the book can also run ``price_grad()`` (ask/bid Greeks
    into a GRAD_DTYPE buffer)."""

    def __init__(self, params, tune=None, greeks=False, graph=False):
        import torch
        self.params = _params(params)
        self.n = len(self.params)
        tune = dict(tune or {})
        if greeks:
            tune["flags"] = int(tune.get("flags", 0)) | BT_TUNE_GREEKS
        if graph:
            tune["flags"] = int(tune.get("flags", 0)) | BT_TUNE_GRAPH
        self.handle = bt_book_create(self.params, tune if tune else None)
        self.out = torch.empty(self.n * RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        self.grad = None

    def info(self):
        return bt_book_info(self.handle)

    def price(self, stream=None):
        bt_book_price(self.handle, self.out.data_ptr(), stream)
        return self.out

    def price_grad(self, stream=None):
        import torch
        if self.grad is None:
            self.grad = torch.empty(self.n * GRAD_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        bt_book_price_grad(self.handle, self.out.data_ptr(), self.grad.data_ptr(), stream)
        return self.out, self.grad

    def price_hedge(self, stream=None):
        """Prices the book and writes the hedges at t = 0 (HEDGE_DTYPE
        records, see hedges())."""
        import torch
        if getattr(self, "hedge", None) is None:
            self.hedge = torch.empty(self.n * HEDGE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        _check(lib().bt_book_price_hedge(self.handle, ctypes.c_void_p(self.out.data_ptr()),
                                         ctypes.c_void_p(self.hedge.data_ptr()), ctypes.c_void_p(_stream_ptr(stream))),
               "bt_book_price_hedge")
        return self.out, self.hedge

    def hedges(self):
        import torch
        torch.cuda.synchronize()
        return np.frombuffer(self.hedge.cpu().numpy().tobytes(), dtype=HEDGE_DTYPE).copy()

    def exercise_offsets(self):
        """Byte offset of each option's exercise maps (n + 1 entries; option
        i's seller plane at off[i], its buyer plane at (off[i] + off[i+1]) / 2)."""
        P = np.zeros(self.n + 1, dtype=np.int64)
        for i, p in enumerate(self.params):
            N = int(p["N"])
            P[i + 1] = (N + 1) * (N + 2) if 1 <= N <= BT_MAX_N else 0
        return np.cumsum(P)

    def price_exercise(self, stream=None):
        """Prices the book and writes the exercise maps of both parties (see
        exercise_maps())."""
        import torch
        off = self.exercise_offsets()
        if getattr(self, "exmap", None) is None or self.exmap.numel() != max(1, int(off[-1])):
            self.exmap = torch.empty(max(1, int(off[-1])), dtype=torch.uint8, device="cuda")
        _check(lib().bt_book_price_exercise(self.handle, ctypes.c_void_p(self.out.data_ptr()),
                                            ctypes.c_void_p(self.exmap.data_ptr()), ctypes.c_void_p(_stream_ptr(stream))),
               "bt_book_price_exercise")
        return self.out, self.exmap

    def exercise_maps(self, i):
        """Option i's maps as a (2, (N+1)(N+2)/2) uint8 array: row 0 the
        seller's, row 1 the buyer's, node (t, c) at t(t+1)/2 + c."""
        import torch
        torch.cuda.synchronize()
        off = self.exercise_offsets()
        return self.exmap[int(off[i]):int(off[i + 1])].cpu().numpy().reshape(2, -1)

    def timings(self):
        return bt_book_timings(self.handle)

    def resolve_overflow(self, stream=None, grad=False):
        """Re-prices overflowed options of the last call; grad=True after
        price_grad() (Greeks re-priced too)."""
        g = self.grad.data_ptr() if grad else 0
        return bt_book_resolve_overflow(self.handle, self.out.data_ptr(), g, stream)

    def results(self):
        import torch
        torch.cuda.synchronize()
        return np.frombuffer(self.out.cpu().numpy().tobytes(), dtype=RESULT_DTYPE).copy()

    def grads(self):
        import torch
        torch.cuda.synchronize()
        return np.frombuffer(self.grad.cpu().numpy().tobytes(), dtype=GRAD_DTYPE).copy()

    def close(self):
        if self.handle is not None:
            bt_book_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def price_book_grad(params, tune=None):
    """Prices a book with Greeks; returns (RESULT_DTYPE, GRAD_DTYPE) arrays."""
    b = Book(params, tune, greeks=True)
    try:
        b.price_grad()
        b.resolve_overflow(grad=True)
        return b.results(), b.grads()
    finally:
        b.close()


def price_book(params, tune=None, resolve=True):
    """Prices a book once and returns the RESULT_DTYPE array; options that
    overflowed the level buffers are re-priced with larger ones unless
    ``resolve`` is False."""
    b = Book(params, tune)
    try:
        b.price()
        if resolve:
            b.resolve_overflow()
        return b.results()
    finally:
        b.close()
