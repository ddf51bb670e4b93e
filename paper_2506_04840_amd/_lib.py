"""ctypes binding of libtucker.so (the C ABI in include/tucker.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. torch supplies device memory and the current stream. If the
library is not built this module raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtucker.so")

MAX_ORDER = 8
MAX_Q = 16
MAX_Q_PVE = 1000
MAX_L = 64
NORM2_WS_BYTES = 8192
NOALLOC_SCRATCH_BYTES = 128 << 20  # TUCKER_NOALLOC_SCRATCH_BYTES

FP64, FP32, BF16 = 0, 1, 2
SHIFT_ADAPTIVE, SHIFT_NONE = 0, 1
POWER_RAW = 1
INFO_NONFINITE, INFO_DEFICIENT, INFO_L_CLAMPED, INFO_INTERNAL = 1, 2, 4, 8

_PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
_SHIFT = {"adaptive": SHIFT_ADAPTIVE, "none": SHIFT_NONE}


class TuckerError(RuntimeError):
    pass


class Shape(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("reserved", ctypes.c_int32), ("dims", ctypes.c_int64 * MAX_ORDER)]


class Info(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_int32),
        ("l", ctypes.c_int32 * MAX_ORDER),
        ("deficient", ctypes.c_int32 * MAX_ORDER),
        ("jacobi_sweeps", ctypes.c_int32),
        ("alpha", (ctypes.c_double * (MAX_Q + 1)) * MAX_ORDER),
        ("sigma_1", (ctypes.c_double * (MAX_Q + 1)) * MAX_ORDER),
        ("sigma_l", (ctypes.c_double * (MAX_Q + 1)) * MAX_ORDER),
        ("normG2", ctypes.c_double),
        ("normA2", ctypes.c_double),
        ("rel_error", ctypes.c_double),
        ("deficient_steps", ctypes.c_int32 * MAX_ORDER),
        ("reserved", ctypes.c_int32 * 6),
    ]


INFO_BYTES = ctypes.sizeof(Info)


class Options(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_int32), ("order_kind", ctypes.c_int32), ("order", ctypes.c_int32 * 8),
                ("holistic", ctypes.c_int32), ("fp32_products", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


OMEGA = {"gaussian": 0, "uniform": 1, "kr_gaussian": 2, "kr_uniform": 3}
ORDER_NATURAL, ORDER_GIVEN, ORDER_DECREASING = 0, 1, 2


FP32_PRODUCTS = {"split": 0, "native": 1}


def make_options(omega: str = "gaussian", order=None, holistic: bool = False,
                 fp32_products: str = "split") -> Options:
    """Options struct: test-matrix kind, processing order (None: 0..d-1,
    "decreasing": by decreasing mode size, or a permutation of the modes), the
    holistic variants of Appendices A / B, and how FP32 solves form their
    products ("split": three-piece BF16 splits on the BF16 matrix cores, the
    default; "native": FP32 matrix-core instructions only)."""
    opt = Options()
    opt.omega = OMEGA[omega]
    opt.holistic = 1 if holistic else 0
    opt.fp32_products = FP32_PRODUCTS[fp32_products]
    if order is None or order == "natural":
        opt.order_kind = ORDER_NATURAL
    elif order == "decreasing":
        opt.order_kind = ORDER_DECREASING
    else:
        perm = [int(k) for k in order]
        if len(perm) > 8:
            raise ValueError("order has more than 8 modes")
        opt.order_kind = ORDER_GIVEN
        for i, k in enumerate(perm):
            opt.order[i] = k
    return opt


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("shape", Shape),
        ("ranks", ctypes.c_int64 * MAX_ORDER),
        ("seed", ctypes.c_uint64),
        ("A", ctypes.c_void_p),
        ("G", ctypes.c_void_p),
        ("U", ctypes.c_void_p * MAX_ORDER),
        ("info", ctypes.c_void_p),
    ]

# Every symbol of include/tucker.h with its ctypes signature.
_P, _I32, _I64, _U64, _SZ, _D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_size_t, ctypes.c_double)
_SHAPE_P = ctypes.POINTER(Shape)
SIGNATURES = {
    "tucker_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tucker_workspace_bytes": (_SZ, [_SHAPE_P, _P, _I32, _I32, ctypes.c_int, _I32]),
    "tucker_workspace_bytes_ex": (_SZ, [_SHAPE_P, _P, _I32, _I32, ctypes.c_int, _I32, _P]),
    "tucker_op_workspace_bytes": (_SZ, [_SHAPE_P, _I32, _I64, ctypes.c_int]),
    "tucker_fill_gaussian": (ctypes.c_int, [_U64, _I32, _I64, _I64, _I64, ctypes.c_int, _P, _P]),
    "tucker_sketch": (ctypes.c_int, [_SHAPE_P, _I32, _P, _I64, _U64, ctypes.c_int, _P, _P, _SZ, _P]),
    "tucker_shifted_power": (ctypes.c_int, [_SHAPE_P, _I32, _P, _I64, _P, _P, _I32, ctypes.c_int, _P, _P, _P, _SZ,
                                            _P]),
    "tucker_orth": (ctypes.c_int, [_I64, _I64, _P, ctypes.c_int, _P, _P, _P, _SZ, _P]),
    "tucker_core": (ctypes.c_int, [_SHAPE_P, _I32, _P, _P, _I64, ctypes.c_int, _P, _P]),
    "tucker_norm2": (ctypes.c_int, [_P, _I64, ctypes.c_int, _P, _P, _SZ, _P]),
    "tucker_rthosvd": (ctypes.c_int, [_SHAPE_P, _P, _P, _I32, _I32, ctypes.c_int, _U64, ctypes.c_int, _P, _P, _P, _P,
                                      _SZ, _P]),
    "tucker_rsthosvd": (ctypes.c_int, [_SHAPE_P, _P, _P, _I32, _I32, ctypes.c_int, _U64, ctypes.c_int, _P, _P, _P, _P,
                                       _SZ, _P]),
    "tucker_rsthosvd_noalloc": (ctypes.c_int, [_SHAPE_P, _P, _P, _I32, _I32, ctypes.c_int, _U64, ctypes.c_int, _P,
                                               _P, _P, _P]),
    "tucker_fill_test_matrix": (ctypes.c_int, [_I32, _U64, _I32, _I32, _P, _I64, _I64, _I64, ctypes.c_int, _P, _P]),
    "tucker_rthosvd_ex": (ctypes.c_int, [_SHAPE_P, _P, _P, _I32, _I32, ctypes.c_int, _U64, ctypes.c_int, _P, _P, _P,
                                         _P, _P, _SZ, _P]),
    "tucker_rsthosvd_ex": (ctypes.c_int, [_SHAPE_P, _P, _P, _I32, _I32, ctypes.c_int, _U64, ctypes.c_int, _P, _P, _P,
                                          _P, _P, _SZ, _P]),
    "tucker_rthosvd_pve": (ctypes.c_int, [_SHAPE_P, _P, _P, _I32, _I32, _D, ctypes.c_int, _U64, ctypes.c_int, _P, _P,
                                          _P, _P, _P, _SZ, _P]),
    "tucker_rsthosvd_pve": (ctypes.c_int, [_SHAPE_P, _P, _P, _I32, _I32, _D, ctypes.c_int, _U64, ctypes.c_int, _P, _P,
                                           _P, _P, _P, _SZ, _P]),
    "tucker_timing_enable": (ctypes.c_int, [_I32, _I32]),
    "tucker_timing_read": (ctypes.c_int, [_I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "tucker_timing_reset": (ctypes.c_int, []),
    "tucker_timing_disable": (ctypes.c_int, []),
    "tucker_batch_plan_bytes": (_SZ, [_I32, _I32, _I32]),
    "tucker_batch_table_bytes": (_SZ, [_I32, _I32, _I32]),
    "tucker_batch_item_bytes": (_SZ, [ctypes.POINTER(BatchItem), _I32, _I32]),
    "tucker_batch_plan": (ctypes.c_int, [_I32, _I32, _I32, _I32, ctypes.POINTER(BatchItem), _I32, _I32, ctypes.c_int,
                                         _P, _SZ, _P, _SZ]),
    "tucker_batch_step": (ctypes.c_int, [_P, _P]),
}

KC = {"colreduce": 0, "rowcontract": 1, "orth": 2, "fill": 3, "reduce": 4, "powerstep": 5}


def _load() -> ctypes.CDLL:
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libtucker.so is not built (python -m paper_2506_04840_amd.build)")
    lib = ctypes.CDLL(_LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(rc: int) -> None:
    if rc == 0:
        return
    msg = lib.tucker_status_string(rc).decode()
    if rc == -1:
        raise ValueError(msg)
    raise TuckerError("tucker status %d: %s" % (rc, msg))


def _shape(dims: Sequence[int]) -> Shape:
    s = Shape()
    s.order = len(dims)  # the library rejects orders above MAX_ORDER
    for k, n in enumerate(list(dims)[:MAX_ORDER]):
        s.dims[k] = int(n)
    return s


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def precision_of(t: torch.Tensor, precision: Optional[str]) -> int:
    if precision is None:
        return FP64 if t.dtype == torch.float64 else FP32
    p = _PREC[precision]
    want = torch.float64 if p == FP64 else torch.float32
    if t.dtype != want:
        raise ValueError("precision %s needs a %s tensor, got %s" % (precision, want, t.dtype))
    return p


def storage_dtype(prec: int) -> torch.dtype:
    return torch.float64 if prec == FP64 else torch.float32


def _dev(t: torch.Tensor, name: str) -> int:
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def workspace_bytes(dims, ranks, p, q, precision: int, sequential: bool, opt: Optional[Options] = None) -> int:
    r = (ctypes.c_int64 * len(ranks))(*[int(x) for x in ranks])
    s = _shape(dims)
    if opt is not None:
        return int(lib.tucker_workspace_bytes_ex(ctypes.byref(s), r, int(p), int(q), precision,
                                                 1 if sequential else 0, ctypes.byref(opt)))
    return int(lib.tucker_workspace_bytes(ctypes.byref(s), r, int(p), int(q), precision, 1 if sequential else 0))


def op_workspace_bytes(dims, mode, l, precision: int) -> int:
    s = _shape(dims)
    return int(lib.tucker_op_workspace_bytes(ctypes.byref(s), int(mode), int(l), precision))


def read_info(info: torch.Tensor) -> dict:
    raw = bytes(info.cpu().numpy().tobytes())
    st = Info.from_buffer_copy(raw)
    return {
        "flags": int(st.flags),
        "l": [int(x) for x in st.l],
        "deficient": [int(x) for x in st.deficient],
        "jacobi_sweeps": int(st.jacobi_sweeps),
        "alpha": [[float(x) for x in row] for row in st.alpha],
        "sigma_1": [[float(x) for x in row] for row in st.sigma_1],
        "sigma_l": [[float(x) for x in row] for row in st.sigma_l],
        "normG2": float(st.normG2),
        "normA2": float(st.normA2),
        "rel_error": float(st.rel_error),
        "deficient_steps": [int(x) for x in st.deficient_steps],
    }


class Solver:
    """A solve configuration with its workspace, reusable across calls.

    The workspace and outputs are allocated once (torch, on the tensor's
    device); run() only enqueues the library's launch sequence.
    """

    def __init__(self, dims, ranks, p=10, q=1, shift="adaptive", seed=1, precision="fp32", sequential=True,
                 device="cuda", omega="gaussian", order=None, holistic=False, fp32_products="split"):
        self.opt = make_options(omega, order, holistic, fp32_products)
        self.plain = (self.opt.omega == 0 and self.opt.order_kind == ORDER_NATURAL and not holistic
                      and self.opt.fp32_products == 0)
        self.dims = tuple(int(x) for x in dims)
        self.ranks = tuple(int(x) for x in ranks)
        self.p, self.q, self.seed = int(p), int(q), int(seed)
        self.prec = _PREC[precision]
        self.shift = _SHIFT[shift]
        self.sequential = bool(sequential)
        self.device = torch.device(device)
        nbytes = workspace_bytes(self.dims, self.ranks, self.p, self.q, self.prec, self.sequential,
                                 None if self.plain else self.opt)
        if nbytes == 0:
            # reproduce the detailed error
            self._call(dry=True)
        dt = storage_dtype(self.prec)
        self.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        self.G = torch.empty(self.ranks, dtype=dt, device=self.device)
        self.U = [torch.empty((n, r), dtype=dt, device=self.device) for n, r in zip(self.dims, self.ranks)]
        self.info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=self.device)
        self._uptr = (ctypes.c_void_p * len(self.U))(*[u.data_ptr() for u in self.U])
        self._shape = _shape(self.dims)
        self._ranks = (ctypes.c_int64 * len(self.ranks))(*self.ranks)

    def _call(self, A: Optional[torch.Tensor] = None, dry: bool = False):
        fn = lib.tucker_rsthosvd if self.sequential else lib.tucker_rthosvd
        if not self.plain:
            fx = lib.tucker_rsthosvd_ex if self.sequential else lib.tucker_rthosvd_ex
            if dry:
                s = _shape(self.dims)
                r = (ctypes.c_int64 * len(self.ranks))(*self.ranks)
                _check(fx(ctypes.byref(s), None, r, self.p, self.q, self.shift, self.seed, self.prec,
                          ctypes.byref(self.opt), None, None, None, None, 0, None))
                return
            _check(fx(ctypes.byref(self._shape), ctypes.c_void_p(A.data_ptr()), self._ranks, self.p, self.q,
                      self.shift, ctypes.c_uint64(self.seed), self.prec, ctypes.byref(self.opt),
                      ctypes.c_void_p(self.G.data_ptr()), self._uptr, ctypes.c_void_p(self.info.data_ptr()),
                      ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_size_t(self.ws.numel()), _stream(self.device)))
            return
        if dry:
            s = _shape(self.dims)
            r = (ctypes.c_int64 * len(self.ranks))(*self.ranks)
            _check(fn(ctypes.byref(s), None, r, self.p, self.q, self.shift, self.seed, self.prec, None, None, None,
                      None, 0, None))
            return
        _check(fn(ctypes.byref(self._shape), ctypes.c_void_p(A.data_ptr()), self._ranks, self.p, self.q, self.shift,
                  ctypes.c_uint64(self.seed), self.prec, ctypes.c_void_p(self.G.data_ptr()), self._uptr,
                  ctypes.c_void_p(self.info.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                  ctypes.c_size_t(self.ws.numel()), _stream(self.device)))

    def run(self, A: torch.Tensor):
        if tuple(A.shape) != self.dims:
            raise ValueError("tensor shape %s != solver dims %s" % (tuple(A.shape), self.dims))
        _dev(A, "A")
        if A.dtype != storage_dtype(self.prec):
            raise ValueError("tensor dtype %s does not match the solver precision" % A.dtype)
        self._call(A)
        return self.G, self.U

    def capture(self, A: torch.Tensor) -> "torch.cuda.CUDAGraph":
        """Record one solve of the tensor at A's address into a HIP graph (the
        library's side streams join the capture through their events); each
        replay() then reruns the whole solve on whatever A holds, into the same
        G, U and info. One eager solve first creates the side streams.

        A T-HOSVD captured this way runs its modes one after another (the
        library does not fork its d - 1 mode streams under capture), with the
        same results as the eager call, whose modes run concurrently."""
        self.run(A)
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(A)
        torch.cuda.synchronize(self.device)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.G, self.U


class PveSolver(Solver):
    """Algorithm 4 (power count per mode by the per-vector-error test): q is
    the largest power count q_max; sequential=False gives its T-HOSVD form
    (Algorithm 2-v3). run() returns after the solve (the library synchronises
    the stream once per power step); q_used holds each q_k."""

    def __init__(self, dims, ranks, p=10, q_max=20, tol=0.5, shift="adaptive", seed=1, precision="fp32",
                 device="cuda", sequential=True):
        if not 1 <= int(q_max) <= MAX_Q_PVE:
            raise ValueError("q_max outside 1..%d" % MAX_Q_PVE)
        super().__init__(dims, ranks, p, min(int(q_max), MAX_Q), shift, seed, precision, sequential, device)
        self.q_max, self.tol = int(q_max), float(tol)
        self._qused = (ctypes.c_int32 * len(self.dims))()

    def capture(self, A: torch.Tensor):
        raise RuntimeError("Algorithm 4 reads its stopping flag on the host after every step: not capturable")

    def _call(self, A: Optional[torch.Tensor] = None, dry: bool = False):
        if dry:
            return super()._call(A, dry)
        fn = lib.tucker_rsthosvd_pve if self.sequential else lib.tucker_rthosvd_pve
        _check(fn(ctypes.byref(self._shape), ctypes.c_void_p(A.data_ptr()), self._ranks, self.p, self.q_max,
                  ctypes.c_double(self.tol), self.shift, ctypes.c_uint64(self.seed), self.prec,
                  ctypes.c_void_p(self.G.data_ptr()), self._uptr, ctypes.c_void_p(self.info.data_ptr()), self._qused,
                  ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_size_t(self.ws.numel()), _stream(self.device)))

    @property
    def q_used(self):
        return [int(x) for x in self._qused]


def rsthosvd_pve(A: torch.Tensor, ranks, p=10, q_max=20, tol=0.5, shift="adaptive", seed=1,
                 precision: Optional[str] = None):
    """Algorithm 4. Returns (G, [U_k], info dict, [q_k])."""
    prec = precision_of(A, precision)
    s = PveSolver(A.shape, ranks, p, q_max, tol, shift, seed, {FP64: "fp64", FP32: "fp32", BF16: "bf16"}[prec],
                  A.device)
    s.run(A.contiguous())
    return s.G, s.U, read_info(s.info), s.q_used


def rthosvd_pve(A: torch.Tensor, ranks, p=10, q_max=20, tol=0.5, shift="adaptive", seed=1,
                precision: Optional[str] = None):
    """Algorithm 4 in the T-HOSVD form (Algorithm 2-v3). Returns (G, [U_k], info dict, [q_k])."""
    prec = precision_of(A, precision)
    s = PveSolver(A.shape, ranks, p, q_max, tol, shift, seed, {FP64: "fp64", FP32: "fp32", BF16: "bf16"}[prec],
                  A.device, sequential=False)
    s.run(A.contiguous())
    return s.G, s.U, read_info(s.info), s.q_used


def rsthosvd(A: torch.Tensor, ranks, p=10, q=1, shift="adaptive", seed=1, precision: Optional[str] = None,
             omega: str = "gaussian", order=None, holistic: bool = False,
             fp32_products: str = "split"):
    """Shifted randomized ST-HOSVD (Algorithm 3). Returns (G, [U_k], info dict)."""
    prec = precision_of(A, precision)
    s = Solver(A.shape, ranks, p, q, shift, seed, {FP64: "fp64", FP32: "fp32", BF16: "bf16"}[prec], True, A.device,
               omega, order, holistic, fp32_products)
    s.run(A.contiguous())
    return s.G, s.U, read_info(s.info)


def rsthosvd_noalloc(A: torch.Tensor, G: torch.Tensor, U: Sequence[torch.Tensor], info: torch.Tensor, ranks, p=10,
                     q=1, shift="adaptive", seed=1, precision: Optional[str] = None) -> None:
    """tucker_rsthosvd_noalloc: Algorithm 3 into caller-allocated G, U_k and
    info, with the library's static device scratch (no workspace)."""
    prec = precision_of(A, precision)
    if not A.is_contiguous():
        raise ValueError("A must be contiguous")
    for t, name in [(A, "A"), (G, "G"), (info, "info")] + [(u, "U[%d]" % k) for k, u in enumerate(U)]:
        _dev(t, name)
    if len(U) != A.dim():
        raise ValueError("one factor per mode")
    uptr = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
    r = (ctypes.c_int64 * len(ranks))(*[int(x) for x in ranks])
    s = _shape(A.shape)
    _check(lib.tucker_rsthosvd_noalloc(ctypes.byref(s), ctypes.c_void_p(A.data_ptr()), r, int(p), int(q),
                                       _SHIFT[shift], ctypes.c_uint64(seed), prec, ctypes.c_void_p(G.data_ptr()),
                                       uptr, ctypes.c_void_p(info.data_ptr()), _stream(A.device)))


def rthosvd(A: torch.Tensor, ranks, p=10, q=1, shift="adaptive", seed=1, precision: Optional[str] = None,
            omega: str = "gaussian", order=None, holistic: bool = False,
            fp32_products: str = "split"):
    """Shifted randomized T-HOSVD (Algorithm 2). Returns (G, [U_k], info dict)."""
    prec = precision_of(A, precision)
    s = Solver(A.shape, ranks, p, q, shift, seed, {FP64: "fp64", FP32: "fp32", BF16: "bf16"}[prec], False, A.device,
               omega, order, holistic, fp32_products)
    s.run(A.contiguous())
    return s.G, s.U, read_info(s.info)


def fill_test_matrix(kind: str, seed: int, mode: int, dims, rows: int, cols: int, precision: str = "fp64",
                     row0: int = 0, device="cuda") -> torch.Tensor:
    """Rows row0 .. row0+rows of test matrix `kind` for mode `mode` of a tensor with sizes `dims`."""
    prec = _PREC[precision]
    out = torch.empty((rows, cols), dtype=storage_dtype(prec), device=device)
    d = (ctypes.c_int64 * len(dims))(*[int(x) for x in dims])
    _check(lib.tucker_fill_test_matrix(OMEGA[kind], ctypes.c_uint64(seed), mode, len(dims), d, row0, rows, cols, prec,
                                       ctypes.c_void_p(out.data_ptr()), _stream(out.device)))
    return out


def fill_gaussian(seed: int, mode: int, rows: int, cols: int, precision: str = "fp64", row0: int = 0,
                  device="cuda") -> torch.Tensor:
    prec = _PREC[precision]
    out = torch.empty((rows, cols), dtype=storage_dtype(prec), device=device)
    _check(lib.tucker_fill_gaussian(ctypes.c_uint64(seed), mode, row0, rows, cols, prec,
                                    ctypes.c_void_p(out.data_ptr()) if out.numel() else None, _stream(out.device)))
    return out


def sketch(X: torch.Tensor, mode: int, l: int, seed: int = 1, precision: Optional[str] = None) -> torch.Tensor:
    """Y = X_(mode) Omega_mode, n x l in the storage dtype (FP64 or FP32)."""
    prec = precision_of(X, precision)
    s = _shape(X.shape)
    Y = torch.empty((X.shape[mode], l), dtype=storage_dtype(prec), device=X.device)
    nbytes = op_workspace_bytes(X.shape, mode, l, prec)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=X.device)
    _check(lib.tucker_sketch(ctypes.byref(s), mode, ctypes.c_void_p(_dev(X, "X")), l, ctypes.c_uint64(seed), prec,
                             ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes,
                             _stream(X.device)))
    return Y


def shifted_power(X: torch.Tensor, mode: int, Q: torch.Tensor, alpha: torch.Tensor, raw: bool = False,
                  precision: Optional[str] = None):
    """One shifted power step. raw: returns M = X_(k)(X_(k)^T Q) - alpha Q (FP64).
    Otherwise returns (Q', Sigma) and updates the device scalar alpha in place."""
    prec = precision_of(X, precision)
    if Q.dtype != storage_dtype(prec) or alpha.dtype != torch.float64:
        raise ValueError("Q must use the storage dtype and alpha must be float64")
    n = X.shape[mode]
    l = Q.shape[1]
    s = _shape(X.shape)
    nbytes = op_workspace_bytes(X.shape, mode, l, prec)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=X.device)
    if raw:
        out = torch.empty((n, l), dtype=torch.float64, device=X.device)
        sigma = None
    else:
        out = torch.empty((n, l), dtype=storage_dtype(prec), device=X.device)
        sigma = torch.empty(l, dtype=torch.float64, device=X.device)
    _check(lib.tucker_shifted_power(ctypes.byref(s), mode, ctypes.c_void_p(_dev(X, "X")), l,
                                    ctypes.c_void_p(_dev(Q, "Q")), ctypes.c_void_p(_dev(alpha, "alpha")),
                                    POWER_RAW if raw else 0, prec, ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(sigma.data_ptr()) if sigma is not None else None,
                                    ctypes.c_void_p(ws.data_ptr()), nbytes, _stream(X.device)))
    return out if raw else (out, sigma)


def orth(Y: torch.Tensor, precision: str = "fp64") -> Tuple[torch.Tensor, torch.Tensor]:
    """[Q, Sigma] = svd(Y, econ) of an FP64 n x l matrix."""
    prec = _PREC[precision]
    if Y.dtype != torch.float64:
        raise ValueError("Y must be float64")
    n, l = Y.shape
    nbytes = op_workspace_bytes((n, max(l, 1)), 0, l, FP64) if l <= min(n, MAX_L) else 0
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=Y.device)
    Q = torch.empty((n, l), dtype=storage_dtype(prec), device=Y.device)
    sigma = torch.empty(l, dtype=torch.float64, device=Y.device)
    _check(lib.tucker_orth(n, l, ctypes.c_void_p(_dev(Y, "Y")), prec, ctypes.c_void_p(Q.data_ptr()),
                           ctypes.c_void_p(sigma.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes,
                           _stream(Y.device)))
    return Q, sigma


def core(X: torch.Tensor, mode: int, U: torch.Tensor, precision: Optional[str] = None) -> torch.Tensor:
    """X x_mode U^T."""
    prec = precision_of(X, precision)
    r = U.shape[1]
    dims = list(X.shape)
    dims[mode] = r
    out = torch.empty(dims, dtype=X.dtype, device=X.device)
    s = _shape(X.shape)
    _check(lib.tucker_core(ctypes.byref(s), mode, ctypes.c_void_p(_dev(X, "X")), ctypes.c_void_p(_dev(U, "U")), r,
                           prec, ctypes.c_void_p(out.data_ptr()), _stream(X.device)))
    return out


def norm2(X: torch.Tensor) -> torch.Tensor:
    prec = FP64 if X.dtype == torch.float64 else FP32
    out = torch.empty(1, dtype=torch.float64, device=X.device)
    ws = torch.empty(NORM2_WS_BYTES, dtype=torch.uint8, device=X.device)
    _check(lib.tucker_norm2(ctypes.c_void_p(_dev(X, "X")), X.numel(), prec, ctypes.c_void_p(out.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), NORM2_WS_BYTES, _stream(X.device)))
    return out


def timing_enable(kernel: str, capacity: int = 4096) -> None:
    _check(lib.tucker_timing_enable(KC[kernel], capacity))


def timing_read(kernel: str) -> dict:
    ms, n, by, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    rc = lib.tucker_timing_read(KC[kernel], ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by), ctypes.byref(fl))
    if rc not in (0, -4):
        _check(rc)
    return {"ms": ms.value, "launches": n.value, "bytes": by.value, "flops": fl.value, "dropped": rc == -4}


def timing_reset() -> None:
    _check(lib.tucker_timing_reset())


def timing_disable() -> None:
    _check(lib.tucker_timing_disable())


# --------------------------------------------------------------------------- batched solves
class BatchSolver:
    """Many small shifted randomized ST-HOSVDs (FP32, one order d, one q) per
    launch sequence. plan(items) writes the pinned plan for a batch (host
    only); step() enqueues the whole batch on the current stream. A step
    captured in a graph replays for later plans (same capacity, d, q, lclass)."""

    def __init__(self, capacity: int, order: int, q: int, p: int, lclass: int, ws_bytes: int,
                 shift: str = "adaptive", device="cuda"):
        self.capacity, self.order, self.q, self.p, self.lclass = int(capacity), int(order), int(q), int(p), int(lclass)
        self.shift = _SHIFT[shift]
        self.device = torch.device(device)
        nb = lib.tucker_batch_plan_bytes(self.capacity, self.order, self.q)
        if nb == 0:
            raise ValueError("bad batch capacity, order or q")
        self.table_bytes = int(lib.tucker_batch_table_bytes(self.capacity, self.order, self.q))
        self.plan_buf = torch.empty(int(nb), dtype=torch.uint8, pin_memory=True)
        self.ws = torch.empty(int(ws_bytes), dtype=torch.uint8, device=self.device)
        self._items = (BatchItem * self.capacity)()

    @staticmethod
    def item(A: torch.Tensor, G: torch.Tensor, U: Sequence[torch.Tensor], ranks, seed: int,
             info: Optional[torch.Tensor] = None) -> BatchItem:
        for t, name in [(A, "A"), (G, "G")] + [(u, "U") for u in U]:
            if t.dtype != torch.float32:
                raise ValueError("batched solves are FP32: %s is %s" % (name, t.dtype))
        it = BatchItem()
        it.shape = _shape(A.shape)
        for k, r in enumerate(ranks):
            it.ranks[k] = int(r)
        it.seed = int(seed)
        it.A = _dev(A, "A")
        it.G = _dev(G, "G")
        for k, u in enumerate(U):
            it.U[k] = _dev(u, "U")
        it.info = info.data_ptr() if info is not None else None
        return it

    def item_bytes(self, it: BatchItem) -> int:
        nb = lib.tucker_batch_item_bytes(ctypes.byref(it), self.p, self.q)
        if nb == 0:
            raise ValueError("invalid batch item")
        return int(nb)

    def plan(self, items: Sequence[BatchItem]) -> None:
        if len(items) > self.capacity:
            raise ValueError("more items than the batch capacity")
        for i, it in enumerate(items):
            self._items[i] = it
        _check(lib.tucker_batch_plan(self.capacity, self.order, self.lclass, len(items), self._items, self.p, self.q,
                                     self.shift,
                                     ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_size_t(self.ws.numel()),
                                     ctypes.c_void_p(self.plan_buf.data_ptr()),
                                     ctypes.c_size_t(self.plan_buf.numel())))

    def step(self) -> None:
        _check(lib.tucker_batch_step(ctypes.c_void_p(self.plan_buf.data_ptr()), _stream(self.device)))

