"""GPU (gfx950) market split solver by lattice enumeration -- Python binding.

A thin ctypes layer over ``libmsp.so`` (C ABI in ``include/msp.h``).  The
functions below carry the C names and only marshal arguments: PyTorch
tensors supply device memory and the current HIP stream, and every step of
the method runs in the library's kernels.  There is no CPU fallback: the
library is loaded on first use, and a missing or unloadable library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsp.so")

MSP_OK = 0
MSP_E_ARG = -1
MSP_E_RANK = -2
MSP_E_NOT_ISOLATED = -3
MSP_E_OVERFLOW = -4
MSP_E_CAPACITY = -5
MSP_E_TIMEOUT = -6
MSP_E_DEVICE = -7
MSP_E_NOMEM = -8
MSP_E_UNSUPPORTED = -9
MSP_E_NUMERIC = -10

MSP_ALL = 0
MSP_FIRST = 1
MSP_LDS = 2
MSP_PLAIN = 0
MSP_LEARNED = 1
MSP_DISCREPANCY = 2
MSP_MAX_N = 127
MSP_NFEAT = 16
MSP_MODEL_NPARAM = 5313

# every symbol include/msp.h declares
EXPORTED = (
    "msp_params_default", "msp_ctx_create", "msp_ctx_destroy", "msp_reduce",
    "msp_gram_schmidt", "msp_enumerate", "msp_solve_batch", "msp_solve_first", "msp_strerror",
    "msp_reduce_bounded", "msp_enumerate_bounded", "msp_autotune", "msp_root_trace", "msp_model_init", "msp_model_set", "msp_model_get", "msp_model_score",
    "msp_model_grad", "msp_train_params_default", "msp_model_train", "msp_reduce_noalloc", "msp_solve_box", "msp_tune_lookup",
)


class MspError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {msp_strerror(code)} ({code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("N", C.c_int64), ("delta", C.c_double), ("eps", C.c_double),
        ("split_depth", C.c_int), ("block", C.c_int), ("target_roots", C.c_int),
        ("hoelder", C.c_int), ("onedir", C.c_int), ("time_cap_ms", C.c_double),
        ("refine", C.c_int), ("refine_keep", C.c_int), ("disc_budget", C.c_int),
        ("bkz_block", C.c_int), ("bkz_tours", C.c_int), ("restarts", C.c_int), ("restart_seed", C.c_uint32),
        ("disc_count", C.c_int), ("root_begin", C.c_int64), ("root_count", C.c_int64),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("evals", C.c_int64), ("nodes", C.c_int64), ("expansions", C.c_int64), ("leaves", C.c_int64),
        ("roots", C.c_int64), ("items", C.c_int64), ("split_depth", C.c_int32), ("k", C.c_int32),
        ("block", C.c_int32), ("pad", C.c_int32),
        ("reduce_ms", C.c_double), ("gs_ms", C.c_double), ("rootgen_ms", C.c_double),
        ("ordering_ms", C.c_double), ("kernel_ms", C.c_double), ("ttfs_ms", C.c_double),
        ("total_ms", C.c_double), ("stages", C.c_int32), ("root_level", C.c_int32),
        ("initial_items", C.c_int64), ("copy", C.c_int32), ("copies", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchDesc(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("A_off", C.c_int64), ("d_off", C.c_int64),
                ("x_off", C.c_int64), ("cap", C.c_int64)]


class TrainParams(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_float), ("pos_weight", C.c_float),
                ("seed", C.c_uint64), ("use_graph", C.c_int)]


class TunePoint(C.Structure):
    _fields_ = [("target_roots", C.c_int32), ("status", C.c_int32), ("ms", C.c_double)]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_08702_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int, C.c_int64
    lib.msp_params_default.argtypes = [C.POINTER(Params)]
    lib.msp_params_default.restype = i32
    lib.msp_ctx_create.argtypes = [i32, C.POINTER(vp)]
    lib.msp_ctx_create.restype = i32
    lib.msp_ctx_destroy.argtypes = [vp]
    lib.msp_ctx_destroy.restype = None
    lib.msp_reduce.argtypes = [vp, i32, i32, vp, vp, C.POINTER(Params), vp, C.POINTER(i32), vp]
    lib.msp_reduce.restype = i32
    lib.msp_gram_schmidt.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    lib.msp_gram_schmidt.restype = i32
    lib.msp_enumerate.argtypes = [vp, i32, i32, vp, vp, vp, i32, i32, i32, C.POINTER(Params), vp, i64,
                                  C.POINTER(i64), C.POINTER(Stats), vp]
    lib.msp_enumerate.restype = i32
    lib.msp_solve_first.argtypes = [vp, i32, i32, vp, vp, i32, C.POINTER(Params), vp, i64, C.POINTER(i64),
                                    C.POINTER(Stats), vp]
    lib.msp_solve_first.restype = i32
    lib.msp_solve_batch.argtypes = [vp, i32, C.POINTER(BatchDesc), vp, vp, i32, i32, C.POINTER(Params), vp,
                                    C.POINTER(i64), C.POINTER(C.c_int32), C.POINTER(Stats), vp]
    lib.msp_solve_batch.restype = i32
    lib.msp_reduce_bounded.argtypes = [vp, i32, i32, vp, vp, vp, C.POINTER(Params), vp, C.POINTER(i32), vp]
    lib.msp_reduce_bounded.restype = i32
    lib.msp_enumerate_bounded.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32, i32, i32, C.POINTER(Params), vp, i64,
                                          C.POINTER(i64), C.POINTER(Stats), vp]
    lib.msp_enumerate_bounded.restype = i32
    lib.msp_solve_box.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32, i32, C.POINTER(Params), vp, i64,
                                  C.POINTER(i64), C.POINTER(Stats), vp]
    lib.msp_solve_box.restype = i32
    lib.msp_autotune.argtypes = [vp, i32, C.POINTER(BatchDesc), vp, vp, i32, i32, C.POINTER(Params),
                                 C.POINTER(Params), C.POINTER(TunePoint), C.POINTER(i32), vp]
    lib.msp_autotune.restype = i32
    lib.msp_tune_lookup.argtypes = [vp, i32, i32, i32, C.POINTER(i32)]
    lib.msp_tune_lookup.restype = i32
    lib.msp_root_trace.argtypes = [vp, i32, i32, vp, vp, vp, i32, C.POINTER(Params), vp, vp, i64,
                                   C.POINTER(i64), C.POINTER(i64), C.POINTER(Stats), vp]
    lib.msp_root_trace.restype = i32
    lib.msp_model_init.argtypes = [vp, C.c_uint64]
    lib.msp_model_init.restype = i32
    lib.msp_model_set.argtypes = [vp, vp]
    lib.msp_model_set.restype = i32
    lib.msp_model_get.argtypes = [vp, vp]
    lib.msp_model_get.restype = i32
    lib.msp_model_score.argtypes = [vp, vp, i64, vp, vp]
    lib.msp_model_score.restype = i32
    lib.msp_model_grad.argtypes = [vp, vp, vp, i64, C.c_float, vp, C.POINTER(C.c_float), vp]
    lib.msp_model_grad.restype = i32
    lib.msp_train_params_default.argtypes = [C.POINTER(TrainParams)]
    lib.msp_train_params_default.restype = i32
    lib.msp_model_train.argtypes = [vp, vp, vp, i64, C.POINTER(TrainParams), vp, vp]
    lib.msp_model_train.restype = i32
    lib.msp_reduce_noalloc.argtypes = [i32, i32, vp, vp, C.POINTER(Params), vp, C.POINTER(i32), vp]
    lib.msp_reduce_noalloc.restype = i32
    lib.msp_strerror.argtypes = [i32]
    lib.msp_strerror.restype = C.c_char_p
    return lib


_LIB: C.CDLL | None = None


def lib() -> C.CDLL:
    """The loaded libmsp (loaded on first call)."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


def msp_strerror(code: int) -> str:
    return lib().msp_strerror(int(code)).decode()


def msp_params_default(**overrides) -> Params:
    p = Params()
    rc = lib().msp_params_default(C.byref(p))
    if rc != MSP_OK:
        raise MspError(rc, "msp_params_default")
    for key, val in overrides.items():
        if not hasattr(p, key):
            raise KeyError(key)
        setattr(p, key, val)
    return p


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_ptr(t: torch.Tensor, dtype: torch.dtype, device: torch.device, name: str) -> int:
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on {device}")
    return t.data_ptr()


# Shape checks, done before any pointer reaches the library: the kernels
# trust the sizes they are given, so a tensor smaller than its stated shape
# would be read or written out of bounds on the device.

def _shape_of(t, name: str) -> tuple:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    return tuple(t.shape)


def _check_instance(A, d) -> tuple[int, int]:
    """A is m x n, d holds m entries; returns (m, n)."""
    sa = _shape_of(A, "A")
    if len(sa) != 2 or sa[0] < 1 or sa[1] < 1:
        raise ValueError(f"A must be a non-empty m x n matrix, got shape {sa}")
    m, n = sa
    sd = _shape_of(d, "d")
    if len(sd) != 1 or sd[0] != m:
        raise ValueError(f"d must hold m = {m} entries, got shape {sd}")
    return m, n


def _check_basis(basis, m: int, n: int) -> int:
    """A kernel basis has n - m + 1 rows of n + 1 entries; returns k."""
    sb = _shape_of(basis, "basis")
    if len(sb) != 2 or sb != (n - m + 1, n + 1):
        raise ValueError(f"basis must have shape ({n - m + 1}, {n + 1}), got {sb}")
    return sb[0]


def _check_out(out, n: int, name: str = "out") -> int:
    """An output buffer holds rows of n bytes; returns its row count."""
    so = _shape_of(out, name)
    if len(so) != 2 or so[1] != n:
        raise ValueError(f"{name} must have n = {n} columns, got shape {so}")
    return so[0]


def _check_bounds(r, n: int, name: str = "r") -> None:
    sr = _shape_of(r, name)
    if len(sr) != 1 or sr[0] != n:
        raise ValueError(f"{name} must hold n = {n} entries, got shape {sr}")


def _check_features(feat, label=None) -> int:
    sf = _shape_of(feat, "feat")
    if len(sf) != 2 or sf[1] != MSP_NFEAT:
        raise ValueError(f"feat must have {MSP_NFEAT} columns, got shape {sf}")
    if label is not None:
        sl = _shape_of(label, "label")
        if len(sl) != 1 or sl[0] != sf[0]:
            raise ValueError(f"label must hold {sf[0]} entries, got shape {sl}")
    return sf[0]


class Context:
    """Owns an ``msp_ctx`` (device workspace) for one device."""

    def __init__(self, device: int | torch.device = 0):
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if dev.type != "cuda":
            raise ValueError("Context needs a GPU device")
        self.device = torch.device("cuda", dev.index if dev.index is not None else 0)
        h = C.c_void_p()
        rc = lib().msp_ctx_create(self.device.index, C.byref(h))
        if rc != MSP_OK:
            raise MspError(rc, "msp_ctx_create")
        self._h = h

    @property
    def handle(self) -> C.c_void_p:
        if self._h is None:
            raise RuntimeError("context destroyed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().msp_ctx_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def msp_ctx_create(device: int = 0) -> Context:
    return Context(device)


def msp_ctx_destroy(ctx: Context) -> None:
    ctx.close()


def msp_gram_schmidt(ctx: Context, basis: torch.Tensor):
    """FP64 Gram-Schmidt of a kernel basis (int64 k x dim on the device).
    Returns (bhat k x dim, mu k x k, beta k) as float64 device tensors."""
    sb = _shape_of(basis, "basis")
    if len(sb) != 2 or sb[0] < 1 or sb[1] < sb[0]:
        raise ValueError(f"basis must be k x dim with 1 <= k <= dim, got shape {sb}")
    k, dim = sb
    dev = ctx.device
    bp = _dev_ptr(basis, torch.int64, dev, "basis")
    bhat = torch.empty((k, dim), dtype=torch.float64, device=dev)
    mu = torch.empty((k, k), dtype=torch.float64, device=dev)
    beta = torch.empty((k,), dtype=torch.float64, device=dev)
    rc = lib().msp_gram_schmidt(ctx.handle, k, dim, bp, bhat.data_ptr(), mu.data_ptr(), beta.data_ptr(),
                               _stream_handle(dev))
    if rc != MSP_OK:
        raise MspError(rc, "msp_gram_schmidt")
    return bhat, mu, beta


def msp_reduce(ctx: Context, A: torch.Tensor, d: torch.Tensor, params: Params | None = None):
    """Embedding + LLL + kernel extraction on the GPU.  Returns the int64
    kernel basis (k x (n+1)) as a device tensor."""
    m, n = _check_instance(A, d)
    dev = ctx.device
    ap = _dev_ptr(A, torch.int32, dev, "A")
    dp = _dev_ptr(d, torch.int64, dev, "d")
    basis = torch.zeros((n + 1, n + 1), dtype=torch.int64, device=dev)
    k = C.c_int(0)
    p = params if params is not None else msp_params_default()
    rc = lib().msp_reduce(ctx.handle, m, n, ap, dp, C.byref(p), basis.data_ptr(), C.byref(k), _stream_handle(dev))
    if rc != MSP_OK:
        raise MspError(rc, "msp_reduce")
    return basis[: k.value].contiguous()


def msp_reduce_noalloc(A: torch.Tensor, d: torch.Tensor, params: Params | None = None,
                       out: torch.Tensor | None = None) -> torch.Tensor:
    """msp_reduce without a context and without any device allocation in the
    library (its scratch is a fixed device array).  Runs on A's device; the
    int64 kernel basis is written to ``out`` ((n+1) x (n+1) rows available,
    allocated here when not given) and returned as its first k rows."""
    m, n = _check_instance(A, d)
    dev = A.device
    if dev.type != "cuda":
        raise ValueError("msp_reduce_noalloc needs device tensors")
    ap = _dev_ptr(A, torch.int32, dev, "A")
    dp = _dev_ptr(d, torch.int64, dev, "d")
    if out is None:
        out = torch.zeros((n + 1, n + 1), dtype=torch.int64, device=dev)
    elif _check_out(out, n + 1, "out") < n + 1:
        raise ValueError(f"out must have n + 1 = {n + 1} rows")
    _dev_ptr(out, torch.int64, dev, "out")
    k = C.c_int(0)
    p = params if params is not None else msp_params_default()
    with torch.cuda.device(dev):
        rc = lib().msp_reduce_noalloc(m, n, ap, dp, C.byref(p), out.data_ptr(), C.byref(k), _stream_handle(dev))
    if rc != MSP_OK:
        raise MspError(rc, "msp_reduce_noalloc")
    return out[: k.value]


@dataclass
class EnumResult:
    x: torch.Tensor       # uint8 (rows, n) on the device, rows = min(n_found, cap)
    n_found: int
    status: int
    stats: dict


def msp_enumerate(ctx: Context, A: torch.Tensor, d: torch.Tensor, basis: torch.Tensor, *,
                  mode: int = MSP_ALL, order: int = MSP_PLAIN, params: Params | None = None,
                  cap: int = 1 << 16, out: torch.Tensor | None = None,
                  raise_on_error: bool = True) -> EnumResult:
    """Enumerate the solutions of A x = d on a given kernel basis.

    MSP_CAPACITY and MSP_TIMEOUT are reported in ``status`` (rows written are
    valid); other errors raise unless ``raise_on_error`` is False."""
    m, n = _check_instance(A, d)
    k = _check_basis(basis, m, n)
    if out is not None:
        cap = min(cap, _check_out(out, n))
    dev = ctx.device
    ap = _dev_ptr(A, torch.int32, dev, "A")
    dp = _dev_ptr(d, torch.int64, dev, "d")
    bp = _dev_ptr(basis, torch.int64, dev, "basis")
    if out is None:
        out = torch.zeros((max(cap, 1), n), dtype=torch.uint8, device=dev)
    else:
        _dev_ptr(out, torch.uint8, dev, "out")
    p = params if params is not None else msp_params_default()
    nf = C.c_int64(0)
    st = Stats()
    rc = lib().msp_enumerate(ctx.handle, m, n, ap, dp, bp, k, int(mode), int(order), C.byref(p),
                            out.data_ptr(), int(cap), C.byref(nf), C.byref(st), _stream_handle(dev))
    if rc not in (MSP_OK, MSP_E_CAPACITY, MSP_E_TIMEOUT) and raise_on_error:
        raise MspError(rc, "msp_enumerate")
    rows = min(nf.value, cap)
    return EnumResult(x=out[:rows], n_found=nf.value, status=rc, stats=st.as_dict())


def msp_solve_first(ctx: Context, A: torch.Tensor, d: torch.Tensor, *, order: int = MSP_PLAIN,
                    params: Params | None = None, cap: int = 64, out: torch.Tensor | None = None,
                    raise_on_error: bool = True) -> EnumResult:
    """A first solution of A x = d by limited discrepancy search over
    params.restarts shuffled copies reduced together (rows in the given
    variable order).  MSP_CAPACITY and MSP_TIMEOUT are reported in ``status``;
    other errors raise unless ``raise_on_error`` is False."""
    m, n = _check_instance(A, d)
    if out is not None:
        cap = min(cap, _check_out(out, n))
    dev = ctx.device
    ap = _dev_ptr(A, torch.int32, dev, "A")
    dp = _dev_ptr(d, torch.int64, dev, "d")
    if out is None:
        out = torch.zeros((max(cap, 1), n), dtype=torch.uint8, device=dev)
    else:
        _dev_ptr(out, torch.uint8, dev, "out")
    p = params if params is not None else msp_params_default()
    nf = C.c_int64(0)
    st = Stats()
    rc = lib().msp_solve_first(ctx.handle, m, n, ap, dp, int(order), C.byref(p), out.data_ptr(), int(cap),
                               C.byref(nf), C.byref(st), _stream_handle(dev))
    if rc not in (MSP_OK, MSP_E_CAPACITY, MSP_E_TIMEOUT) and raise_on_error:
        raise MspError(rc, "msp_solve_first")
    rows = min(nf.value, cap)
    return EnumResult(x=out[:rows], n_found=nf.value, status=rc, stats=st.as_dict())


@dataclass
class BatchResult:
    x: list           # per instance: uint8 (rows, n) device tensor (views into one packed buffer)
    n_found: list     # per instance
    status: list      # per instance MSP_* code
    stats: list       # per instance dict
    rc: int           # MSP_OK, or the first non-OK instance status


def _pack(ctx: Context, As: list, ds: list, cap: int):
    if len(As) != len(ds) or not As:
        raise ValueError("As and ds must be non-empty lists of equal length")
    dev = ctx.device
    for i, (A, d) in enumerate(zip(As, ds)):
        try:
            _check_instance(A, d)
        except ValueError as e:
            raise ValueError(f"instance {i}: {e}") from None
        _dev_ptr(A, torch.int32, dev, f"As[{i}]")
        _dev_ptr(d, torch.int64, dev, f"ds[{i}]")
    b = len(As)
    desc = (BatchDesc * b)()
    a_off = d_off = x_off = 0
    for i, A in enumerate(As):
        m, n = A.shape
        desc[i] = BatchDesc(m, n, a_off, d_off, x_off, cap)
        a_off += m * n
        d_off += m
        x_off += cap * n
    A_all = torch.cat([A.reshape(-1) for A in As])
    d_all = torch.cat([d.reshape(-1) for d in ds])
    return desc, A_all, d_all, x_off


def msp_autotune(ctx: Context, As: list, ds: list, *, mode: int = MSP_ALL, order: int = MSP_PLAIN,
                 params: Params | None = None):
    """Pick target_roots on tuning instances; returns (best Params, [(target_roots, status, ms), ...])."""
    desc, A_all, d_all, _ = _pack(ctx, As, ds, 0)
    p = params if params is not None else msp_params_default()
    best = Params()
    pts = (TunePoint * 8)()
    npts = C.c_int(0)
    rc = lib().msp_autotune(ctx.handle, len(As), desc, A_all.data_ptr(), d_all.data_ptr(), int(mode), int(order),
                            C.byref(p), C.byref(best), pts, C.byref(npts), _stream_handle(ctx.device))
    if rc != MSP_OK:
        raise MspError(rc, "msp_autotune")
    return best, [(pts[i].target_roots, pts[i].status, pts[i].ms) for i in range(npts.value)]


def msp_tune_lookup(ctx: Context, m: int, n: int, *, mode: int = MSP_ALL) -> int:
    """Root count msp_autotune chose for shape (m, n) in this context (0: not tuned)."""
    t = C.c_int(0)
    rc = lib().msp_tune_lookup(ctx.handle, int(mode), int(m), int(n), C.byref(t))
    if rc != MSP_OK:
        raise MspError(rc, "msp_tune_lookup")
    return t.value


def msp_solve_batch(ctx: Context, As: list, ds: list, *, mode: int = MSP_ALL, order: int = MSP_PLAIN,
                    params: Params | None = None, cap: int = 1024) -> BatchResult:
    """Reduce and enumerate a batch of instances of uneven shape.

    As / ds: lists of int32 (m_i x n_i) and int64 (m_i) device tensors.  They
    are packed into one buffer each (plain device copies) and described to
    the library by element offsets; every instance gets ``cap`` output rows."""
    dev = ctx.device
    desc, A_all, d_all, x_off = _pack(ctx, As, ds, cap)
    b = len(As)
    x_all = torch.zeros(max(x_off, 1), dtype=torch.uint8, device=dev)
    nf = (C.c_int64 * b)()
    st = (C.c_int32 * b)()
    stats = (Stats * b)()
    p = params if params is not None else msp_params_default()
    rc = lib().msp_solve_batch(ctx.handle, b, desc, A_all.data_ptr(), d_all.data_ptr(), int(mode), int(order),
                               C.byref(p), x_all.data_ptr(), nf, st, stats, _stream_handle(dev))
    if rc == MSP_E_ARG or rc == MSP_E_DEVICE or rc == MSP_E_NOMEM:
        raise MspError(rc, "msp_solve_batch")
    xs = []
    for i in range(b):
        n = desc[i].n
        rows = min(nf[i], cap)
        xs.append(x_all[desc[i].x_off: desc[i].x_off + cap * n].view(cap, n)[:rows])
    return BatchResult(x=xs, n_found=list(nf), status=list(st), stats=[s.as_dict() for s in stats], rc=rc)


# ---- root traces and the root-scoring model ---------------------------------

@dataclass
class Trace:
    feat: torch.Tensor    # float32 (roots, MSP_NFEAT) on the device
    label: torch.Tensor   # uint8 (roots,) on the device: 1 iff a solution lies below the root
    n_found: int
    stats: dict


def msp_root_trace(ctx: Context, A: torch.Tensor, d: torch.Tensor, basis: torch.Tensor, *,
                   params: Params | None = None, cap_roots: int = 1 << 20) -> Trace:
    """Exhaustive enumeration that also returns per-root features and labels."""
    m, n = _check_instance(A, d)
    k = _check_basis(basis, m, n)
    dev = ctx.device
    ap = _dev_ptr(A, torch.int32, dev, "A")
    dp = _dev_ptr(d, torch.int64, dev, "d")
    bp = _dev_ptr(basis, torch.int64, dev, "basis")
    p = params if params is not None else msp_params_default()
    for _ in range(2):
        feat = torch.empty((max(cap_roots, 1), MSP_NFEAT), dtype=torch.float32, device=dev)
        label = torch.empty((max(cap_roots, 1),), dtype=torch.uint8, device=dev)
        nr, nf, st = C.c_int64(0), C.c_int64(0), Stats()
        rc = lib().msp_root_trace(ctx.handle, m, n, ap, dp, bp, k, C.byref(p), feat.data_ptr(), label.data_ptr(),
                                  int(cap_roots), C.byref(nr), C.byref(nf), C.byref(st), _stream_handle(dev))
        if rc == MSP_E_CAPACITY and nr.value > cap_roots:
            cap_roots = nr.value  # more roots than room: run again with room for all
            continue
        if rc != MSP_OK:
            raise MspError(rc, "msp_root_trace")
        return Trace(feat=feat[: nr.value], label=label[: nr.value], n_found=nf.value, stats=st.as_dict())
    raise MspError(MSP_E_CAPACITY, "msp_root_trace")


def msp_model_init(ctx: Context, seed: int = 0) -> None:
    rc = lib().msp_model_init(ctx.handle, int(seed))
    if rc != MSP_OK:
        raise MspError(rc, "msp_model_init")


def msp_model_set(ctx: Context, w) -> None:
    import numpy as np
    w = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
    if w.size != MSP_MODEL_NPARAM:
        raise ValueError(f"expected {MSP_MODEL_NPARAM} parameters, got {w.size}")
    rc = lib().msp_model_set(ctx.handle, w.ctypes.data)
    if rc != MSP_OK:
        raise MspError(rc, "msp_model_set")


def msp_model_get(ctx: Context):
    import numpy as np
    w = np.empty(MSP_MODEL_NPARAM, dtype=np.float32)
    rc = lib().msp_model_get(ctx.handle, w.ctypes.data)
    if rc != MSP_OK:
        raise MspError(rc, "msp_model_get")
    return w


def msp_model_score(ctx: Context, feat: torch.Tensor) -> torch.Tensor:
    count = _check_features(feat)
    dev = ctx.device
    fp = _dev_ptr(feat, torch.float32, dev, "feat")
    logit = torch.empty((count,), dtype=torch.float32, device=dev)
    rc = lib().msp_model_score(ctx.handle, fp, count, logit.data_ptr(), _stream_handle(dev))
    if rc != MSP_OK:
        raise MspError(rc, "msp_model_score")
    return logit


def msp_model_grad(ctx: Context, feat: torch.Tensor, label: torch.Tensor, pos_weight: float = 1.0):
    """Returns (gradient as a float32 device tensor, loss)."""
    _check_features(feat, label)
    dev = ctx.device
    fp = _dev_ptr(feat, torch.float32, dev, "feat")
    lp = _dev_ptr(label, torch.uint8, dev, "label")
    grad = torch.empty((MSP_MODEL_NPARAM,), dtype=torch.float32, device=dev)
    loss = C.c_float(0.0)
    rc = lib().msp_model_grad(ctx.handle, fp, lp, feat.shape[0], float(pos_weight), grad.data_ptr(),
                              C.byref(loss), _stream_handle(dev))
    if rc != MSP_OK:
        raise MspError(rc, "msp_model_grad")
    return grad, loss.value


def msp_train_params_default(**overrides) -> TrainParams:
    tp = TrainParams()
    rc = lib().msp_train_params_default(C.byref(tp))
    if rc != MSP_OK:
        raise MspError(rc, "msp_train_params_default")
    for key, val in overrides.items():
        if not hasattr(tp, key):
            raise KeyError(key)
        setattr(tp, key, val)
    return tp


def msp_model_train(ctx: Context, feat: torch.Tensor, label: torch.Tensor, tp: TrainParams | None = None):
    """Train the context's model on (feat, label); returns the per-epoch losses."""
    _check_features(feat, label)
    dev = ctx.device
    fp = _dev_ptr(feat, torch.float32, dev, "feat")
    lp = _dev_ptr(label, torch.uint8, dev, "label")
    tp = tp if tp is not None else msp_train_params_default()
    losses = (C.c_float * max(1, tp.epochs))()
    rc = lib().msp_model_train(ctx.handle, fp, lp, feat.shape[0], C.byref(tp), losses, _stream_handle(dev))
    if rc != MSP_OK:
        raise MspError(rc, "msp_model_train")
    return list(losses)[: tp.epochs]


# ---- bounded variables ------------------------------------------------------

def msp_reduce_bounded(ctx: Context, A: torch.Tensor, d: torch.Tensor, r: torch.Tensor,
                       params: Params | None = None) -> torch.Tensor:
    """Embedding with upper bounds r (int32 device tensor, 1..255) + LLL +
    kernel extraction; returns the int64 kernel basis (k x (n+1))."""
    m, n = _check_instance(A, d)
    _check_bounds(r, n)
    dev = ctx.device
    ap = _dev_ptr(A, torch.int32, dev, "A")
    dp = _dev_ptr(d, torch.int64, dev, "d")
    rp = _dev_ptr(r, torch.int32, dev, "r")
    basis = torch.zeros((n + 1, n + 1), dtype=torch.int64, device=dev)
    k = C.c_int(0)
    p = params if params is not None else msp_params_default()
    rc = lib().msp_reduce_bounded(ctx.handle, m, n, ap, dp, rp, C.byref(p), basis.data_ptr(), C.byref(k),
                                  _stream_handle(dev))
    if rc != MSP_OK:
        raise MspError(rc, "msp_reduce_bounded")
    return basis[: k.value].contiguous()


def msp_enumerate_bounded(ctx: Context, A: torch.Tensor, d: torch.Tensor, r: torch.Tensor, basis: torch.Tensor, *,
                          mode: int = MSP_ALL, order: int = MSP_PLAIN, params: Params | None = None,
                          cap: int = 1 << 16, raise_on_error: bool = True) -> EnumResult:
    """All (or the first) x with A x = d and 0 <= x <= r on a given kernel basis."""
    m, n = _check_instance(A, d)
    _check_bounds(r, n)
    k = _check_basis(basis, m, n)
    dev = ctx.device
    ap = _dev_ptr(A, torch.int32, dev, "A")
    dp = _dev_ptr(d, torch.int64, dev, "d")
    rp = _dev_ptr(r, torch.int32, dev, "r")
    bp = _dev_ptr(basis, torch.int64, dev, "basis")
    out = torch.zeros((max(cap, 1), n), dtype=torch.uint8, device=dev)
    p = params if params is not None else msp_params_default()
    nf = C.c_int64(0)
    st = Stats()
    rc = lib().msp_enumerate_bounded(ctx.handle, m, n, ap, dp, rp, bp, k, int(mode), int(order), C.byref(p),
                                     out.data_ptr(), int(cap), C.byref(nf), C.byref(st), _stream_handle(dev))
    if rc not in (MSP_OK, MSP_E_CAPACITY, MSP_E_TIMEOUT) and raise_on_error:
        raise MspError(rc, "msp_enumerate_bounded")
    rows = min(nf.value, cap)
    return EnumResult(x=out[:rows], n_found=nf.value, status=rc, stats=st.as_dict())


def msp_solve_box(ctx: Context, A: torch.Tensor, d: torch.Tensor, lo: torch.Tensor, hi: torch.Tensor, *,
                  mode: int = MSP_ALL, order: int = MSP_PLAIN, params: Params | None = None,
                  cap: int = 1 << 16, raise_on_error: bool = True) -> EnumResult:
    """All (or the first) integer x with A x = d and lo <= x <= hi (int32
    device tensors of n entries, 1 <= hi - lo <= 255); rows are int32."""
    m, n = _check_instance(A, d)
    _check_bounds(lo, n, "lo")
    _check_bounds(hi, n, "hi")
    dev = ctx.device
    ap = _dev_ptr(A, torch.int32, dev, "A")
    dp = _dev_ptr(d, torch.int64, dev, "d")
    lp = _dev_ptr(lo, torch.int32, dev, "lo")
    hp = _dev_ptr(hi, torch.int32, dev, "hi")
    out = torch.zeros((max(cap, 1), n), dtype=torch.int32, device=dev)
    p = params if params is not None else msp_params_default()
    nf = C.c_int64(0)
    st = Stats()
    rc = lib().msp_solve_box(ctx.handle, m, n, ap, dp, lp, hp, int(mode), int(order), C.byref(p), out.data_ptr(),
                             int(cap), C.byref(nf), C.byref(st), _stream_handle(dev))
    if rc not in (MSP_OK, MSP_E_CAPACITY, MSP_E_TIMEOUT) and raise_on_error:
        raise MspError(rc, "msp_solve_box")
    rows = min(nf.value, cap)
    return EnumResult(x=out[:rows], n_found=nf.value, status=rc, stats=st.as_dict())
