"""Per-pixel Kronecker STAP on AMD MI355X: thin Python binding of libkstap.so.

Argument marshalling only: every step of the pass runs in the library's HIP
kernels.  PyTorch tensors supply device memory and the HIP stream.

    plan = kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4)
    T, D = kstap.run(plan, x)          # x: torch.complex64 [p, H, W, q] on a GPU

The C ABI is declared in include/kstap.h; the names here mirror it.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkstap.so")

STAP_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY", 4: "DEVICE", 5: "BUSY",
                6: "INTERNAL"}
PRECISIONS = {"fp32": 0, "bf16x3": 1, "fp32_f64": 2}
STAT_MODES = {"glrt": 0, "fixed": 1}
FILTERS = {"kron": 0, "classical": 1}


class StapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class StapConfig(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int32), ("q", ctypes.c_int32), ("n", ctypes.c_int32),
        ("stencil", ctypes.POINTER(ctypes.c_int32)),
        ("window", ctypes.c_int32), ("guard", ctypes.c_int32),
        ("r_a", ctypes.c_int32), ("r_b", ctypes.c_int32),
        ("eps", ctypes.c_double), ("min_iter", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("stat_mode", ctypes.c_int32),
        ("b_steer", ctypes.POINTER(ctypes.c_float)), ("h_steer", ctypes.POINTER(ctypes.c_float)),
        ("tau", ctypes.c_double), ("pfa", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("filter", ctypes.c_int32), ("nbank", ctypes.c_int32), ("passes", ctypes.c_int32),
    ]


class StapLrkConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32), ("r_a", ctypes.c_int32),
                ("eps", ctypes.c_double), ("min_iter", ctypes.c_int32), ("max_iter", ctypes.c_int32)]


class StapLrstapConfig(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double)]


class StapTrueCov(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("q", ctypes.c_int32), ("ra", ctypes.c_int32), ("rb", ctypes.c_int32),
                ("UA", ctypes.c_void_p), ("lamA", ctypes.c_void_p), ("UB", ctypes.c_void_p), ("lamB", ctypes.c_void_p),
                ("sigma2", ctypes.c_double), ("tau2", ctypes.c_double)]


class StapFilterSet(ctypes.Structure):
    _fields_ = [("filter", ctypes.c_int32), ("npix", ctypes.c_int32), ("r_a", ctypes.c_int32), ("r_b", ctypes.c_int32),
                ("r", ctypes.c_int32), ("UA", ctypes.c_void_p), ("UB", ctypes.c_void_p), ("U", ctypes.c_void_p)]


SINR_FILTERS = {"kron": 0, "classical": 1, "lrstap": 2}


class StapOutputs(ctypes.Structure):
    _fields_ = [("T", ctypes.c_void_p), ("D", ctypes.c_void_p), ("E", ctypes.c_void_p), ("bin", ctypes.c_void_p),
                ("Tpass", ctypes.c_void_p), ("C", ctypes.c_void_p)]


class StapProbeOut(ctypes.Structure):
    _fields_ = [("UA", ctypes.c_void_p), ("UB", ctypes.c_void_p), ("eta", ctypes.c_void_p),
                ("iters", ctypes.c_void_p), ("T", ctypes.c_void_p)]


class StapTile(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("x", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("T", ctypes.c_void_p), ("D", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libkstap.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1604_03622_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i32, p_ = ctypes.c_int32, ctypes.c_void_p
    sigs = {
        "stap_config_default": [ctypes.POINTER(StapConfig)],
        "stap_plan_create": [ctypes.POINTER(StapConfig), ctypes.POINTER(p_)],
        "stap_plan": [ctypes.POINTER(StapConfig), ctypes.POINTER(p_)],
        "stap_plan_destroy": [p_],
        "stap_plan_info": [p_, ctypes.POINTER(ctypes.c_double)] + [ctypes.POINTER(i32)] * 5,
        "stap_plan_stencil": [p_, ctypes.POINTER(i32)],
        "stap_valid_region": [p_, i32, i32] + [ctypes.POINTER(i32)] * 4,
        "stap_plan_order": [p_, i32, i32, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "stap_plan_moves": [p_, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                            ctypes.POINTER(i32)],
        "stap_run": [p_, p_, i32, i32, p_, p_, p_],
        "stap_run_ex": [p_, p_, i32, i32, ctypes.POINTER(StapOutputs), p_],
        "stap_lrkron": [ctypes.POINTER(StapLrkConfig), p_, p_, p_, p_, p_],
        "stap_run_noalloc": [p_, p_, i32, i32, p_, p_, p_],
        "stap_probe": [p_, p_, i32, i32, p_, i32, ctypes.POINTER(StapProbeOut), p_],
        "stap_lrstap_probe": [p_, ctypes.POINTER(StapLrstapConfig), p_, i32, i32, p_, i32, p_, p_, p_, p_, p_],
        "stap_sinr_loss": [ctypes.POINTER(StapTrueCov), ctypes.POINTER(StapFilterSet), p_, i32, p_, i32, p_, p_],
        "stap_run_batch": [ctypes.POINTER(StapTile), i32, p_],
        "stap_batch_create": [ctypes.POINTER(StapTile), i32, i32, ctypes.POINTER(p_)],
        "stap_batch_launch": [p_, p_],
        "stap_batch_tune": [p_, p_, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)],
        "stap_batch_info": [p_, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                            ctypes.POINTER(i32)],
        "stap_batch_destroy": [p_],
        "stap_batch_class_info": [p_, i32] + [ctypes.POINTER(i32)] * 6,
        "stap_tune_lookup": [ctypes.c_char_p, i32, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                             ctypes.POINTER(i32)],
        "stap_tune_record": [ctypes.c_char_p, i32, i32, i32, i32, i32, i32, ctypes.c_double],
        "stap_server_create": [ctypes.c_size_t, i32, ctypes.c_int64, ctypes.POINTER(p_)],
        "stap_server_submit": [p_, p_, p_, i32, i32, i32, p_, p_, p_, ctypes.POINTER(ctypes.c_uint64)],
        "stap_server_wait": [p_, ctypes.c_uint64, i32, ctypes.POINTER(ctypes.c_double)],
        "stap_server_stats": [p_, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
        "stap_server_destroy": [p_],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.stap_last_error.restype = ctypes.c_char_p
    L.stap_last_error.argtypes = []
    L.stap_version.restype = ctypes.c_char_p
    L.stap_version.argtypes = []
    _lib = L
    return L


def _check(status: int) -> None:
    if status != STAP_OK:
        raise StapError(status, lib().stap_last_error().decode())


def _cfloat_array(values, count: int):
    arr = np.ascontiguousarray(np.asarray(values, dtype=np.complex64).reshape(count))
    buf = (ctypes.c_float * (2 * count))(*arr.view(np.float32).tolist())
    return buf


class Plan:
    """An immutable detector plan (host only; usable on any device/stream)."""

    def __init__(self, p: int, q: int, n: int, r_a: int = 1, r_b: int = 3,
                 stencil: Optional[Sequence] = None, window: int = 0, guard: int = 3,
                 eps: float = 1e-6, min_iter: int = 2, max_iter: int = 50,
                 stat_mode: str = "glrt", b_steer=None, h_steer=None,
                 tau: float = 0.0, pfa: float = 1e-4, precision: str = "fp32", filter: str = "kron",
                 nbank: int = 0, passes: int = 1):
        L = lib()
        cfg = StapConfig()
        _check(L.stap_config_default(ctypes.byref(cfg)))
        cfg.p, cfg.q, cfg.n = p, q, n
        cfg.window, cfg.guard = window, guard
        cfg.r_a, cfg.r_b = r_a, r_b
        cfg.eps, cfg.min_iter, cfg.max_iter = eps, min_iter, max_iter
        cfg.stat_mode = STAT_MODES[stat_mode]
        cfg.tau, cfg.pfa = tau, pfa
        cfg.precision = PRECISIONS[precision]
        cfg.filter = FILTERS[filter]
        cfg.nbank = nbank
        cfg.passes = passes
        keep = []
        if stencil is not None:
            st = np.ascontiguousarray(np.asarray(stencil, dtype=np.int32).reshape(-1))
            buf = (ctypes.c_int32 * st.size)(*st.tolist())
            keep.append(buf)
            cfg.stencil = ctypes.cast(buf, ctypes.POINTER(ctypes.c_int32))
        if b_steer is not None:
            buf = _cfloat_array(b_steer, q)
            keep.append(buf)
            cfg.b_steer = ctypes.cast(buf, ctypes.POINTER(ctypes.c_float))
        if h_steer is not None:
            buf = _cfloat_array(h_steer, p)
            keep.append(buf)
            cfg.h_steer = ctypes.cast(buf, ctypes.POINTER(ctypes.c_float))
        handle = ctypes.c_void_p()
        _check(L.stap_plan_create(ctypes.byref(cfg), ctypes.byref(handle)))
        self._h = handle
        self.p, self.q, self.n, self.r_a, self.r_b = p, q, n, r_a, r_b
        self.precision = precision
        self.filter, self.nbank, self.passes = filter, nbank, passes
        tau_v = ctypes.c_double()
        ints = [ctypes.c_int32() for _ in range(5)]
        _check(L.stap_plan_info(self._h, ctypes.byref(tau_v), *[ctypes.byref(v) for v in ints]))
        self.tau = tau_v.value
        self.window = ints[0].value
        self.extent = tuple(v.value for v in ints[1:])
        st = (ctypes.c_int32 * (2 * n))()
        _check(L.stap_plan_stencil(self._h, st))
        self.stencil = np.frombuffer(st, dtype=np.int32).reshape(n, 2).copy()

    @property
    def handle(self):
        return self._h

    def valid_region(self, H: int, W: int):
        out = [ctypes.c_int32() for _ in range(4)]
        _check(lib().stap_valid_region(self._h, H, W, *[ctypes.byref(v) for v in out]))
        return tuple(v.value for v in out)

    def order(self, H: int, W: int, first: int = 0, count: int = None):
        """Visiting order of stap_run: (pix [count, 2] with (-1, -1) past the
        edge, move [count]: 0 right, 1 left, 2 down, -1 a chain start)."""
        if count is None:
            count = ((H + 3) // 4) * ((W + 3) // 4) * 16 - first
        pix = np.empty((count, 2), dtype=np.int32)
        mv = np.empty(count, dtype=np.int32)
        p32 = ctypes.POINTER(ctypes.c_int32)
        _check(lib().stap_plan_order(self._h, H, W, first, count, pix.ctypes.data_as(p32), mv.ctypes.data_as(p32)))
        return pix, mv

    def moves(self, move: int):
        """Offsets (dr, dc) entering and leaving the stencil on a one-pixel
        move (0 right, 1 left, 2 down), or None if the plan never slides."""
        na, nr = ctypes.c_int32(), ctypes.c_int32()
        add = np.zeros((48, 2), dtype=np.int32)
        rem = np.zeros((48, 2), dtype=np.int32)
        p32 = ctypes.POINTER(ctypes.c_int32)
        _check(lib().stap_plan_moves(self._h, move, ctypes.byref(na), ctypes.byref(nr), add.ctypes.data_as(p32),
                                     rem.ctypes.data_as(p32)))
        if na.value < 0:
            return None
        return add[:na.value].copy(), rem[:nr.value].copy()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.stap_plan_destroy(h)
            self._h = None


def _stream_handle(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_frame(plan: Plan, x):
    import torch
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex64 or not x.is_cuda:
        raise TypeError("x must be a torch.complex64 tensor on a GPU")
    if x.dim() != 4 or x.shape[0] != plan.p or x.shape[3] != plan.q:
        raise ValueError(f"x must have shape [p={plan.p}, H, W, q={plan.q}], got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError("x must be contiguous")
    return int(x.shape[1]), int(x.shape[2])


def run(plan: Plan, x, T=None, D=None, stream=None, with_detections: bool = True):
    """Whole-frame pass; returns (T float32 [H, W], D uint8 [H, W] or None).
    Asynchronous on `stream` (default: torch's current stream)."""
    import torch
    H, W = _check_frame(plan, x)
    if T is None:
        T = torch.empty((H, W), dtype=torch.float32, device=x.device)
    if D is None and with_detections:
        D = torch.empty((H, W), dtype=torch.uint8, device=x.device)
    _check(lib().stap_run(plan.handle, ctypes.c_void_p(x.data_ptr()), H, W, ctypes.c_void_p(T.data_ptr()),
                          ctypes.c_void_p(D.data_ptr()) if D is not None else None, _stream_handle(stream)))
    return T, D


def run_ex(plan: Plan, x, enhancement: bool = True, bins: bool = True, stream=None) -> dict:
    """Whole-frame pass with the optional outputs of stap_run_ex: T, D, the
    enhancement image E, the Doppler bin of the maximum, and for multipass
    plans the per-pass images T_pass [K, H, W] and change images C [K-1, H, W]."""
    import torch
    H, W = _check_frame(plan, x)
    dev = x.device
    out = dict(T=torch.empty((H, W), dtype=torch.float32, device=dev),
               D=torch.empty((H, W), dtype=torch.uint8, device=dev),
               E=torch.empty((H, W), dtype=torch.float32, device=dev) if enhancement else None,
               bin=torch.empty((H, W), dtype=torch.uint8, device=dev) if bins else None)
    if plan.passes > 1:
        out["T_pass"] = torch.empty((plan.passes, H, W), dtype=torch.float32, device=dev)
        out["C"] = torch.empty((plan.passes - 1, H, W), dtype=torch.float32, device=dev)
    ptr = lambda name: out[name].data_ptr() if out.get(name) is not None else None  # noqa: E731
    so = StapOutputs(ptr("T"), ptr("D"), ptr("E"), ptr("bin"), ptr("T_pass"), ptr("C"))
    _check(lib().stap_run_ex(plan.handle, ctypes.c_void_p(x.data_ptr()), H, W, ctypes.byref(so),
                             _stream_handle(stream)))
    return out


def lrkron(X, r_a: int = 1, eps: float = 1e-6, min_iter: int = 2, max_iter: int = 50, with_B: bool = True,
           stream=None) -> dict:
    """stap_lrkron: LR-Kron on the covariance of the snapshots X
    (torch.complex64 [n, p, q] on a GPU).  Returns A [p, p], B [q, q] (or
    None) and stats (float64: eta, iterations, ||R||_F, ||b||)."""
    import torch
    if not isinstance(X, torch.Tensor) or X.dtype != torch.complex64 or not X.is_cuda or X.dim() != 3:
        raise TypeError("X must be a torch.complex64 tensor [n, p, q] on a GPU")
    X = X.contiguous()
    n, p, q = (int(v) for v in X.shape)
    dev = X.device
    A = torch.empty((p, p), dtype=torch.complex64, device=dev)
    B = torch.empty((q, q), dtype=torch.complex64, device=dev) if with_B else None
    stats = torch.empty(4, dtype=torch.float64, device=dev)
    cfg = StapLrkConfig(n, p, q, r_a, eps, min_iter, max_iter)
    _check(lib().stap_lrkron(ctypes.byref(cfg), ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(A.data_ptr()),
                             ctypes.c_void_p(B.data_ptr()) if B is not None else None,
                             ctypes.c_void_p(stats.data_ptr()), _stream_handle(stream)))
    return dict(A=A, B=B, stats=stats, _keep=X)


NOALLOC_MAX_BYTES = 128 << 20


def run_noalloc(plan: Plan, x, T, D=None, stream=None):
    """stap_run_noalloc: the whole-frame pass into caller-provided T (float32
    [H, W]) and D (uint8 [H, W] or None), with no device allocation in the
    library (the mixed path's planes use a static per-device work area of
    NOALLOC_MAX_BYTES; calls that overlap on one device race)."""
    import torch
    H, W = _check_frame(plan, x)
    for name, t, dt in (("T", T, torch.float32), ("D", D, torch.uint8)):
        if t is None and name == "D":
            continue
        if not isinstance(t, torch.Tensor) or t.dtype != dt or t.device != x.device or tuple(t.shape) != (H, W) \
                or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} tensor [H, W] on the frame's device")
    _check(lib().stap_run_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), H, W, ctypes.c_void_p(T.data_ptr()),
                                  ctypes.c_void_p(D.data_ptr()) if D is not None else None, _stream_handle(stream)))
    return T, D


def probe(plan: Plan, x, pix, stream=None) -> dict:
    """Per-pixel pass with intermediates for pixels pix [(r, c), ...]."""
    import torch
    H, W = _check_frame(plan, x)
    dev = x.device
    pix_t = torch.as_tensor(np.asarray(pix, dtype=np.int32).reshape(-1, 2), device=dev).contiguous()
    npix = int(pix_t.shape[0])
    out = dict(
        T=torch.empty(npix, dtype=torch.float32, device=dev),
        eta=torch.empty(npix, dtype=torch.float32, device=dev),
        iters=torch.empty(npix, dtype=torch.int32, device=dev),
        U_A=torch.empty((npix, plan.p, plan.r_a), dtype=torch.complex64, device=dev),
        U_B=torch.empty((npix, plan.q, max(plan.r_b, 0)), dtype=torch.complex64, device=dev),
    )
    po = StapProbeOut(out["U_A"].data_ptr(), out["U_B"].data_ptr() if plan.r_b > 0 else None,
                      out["eta"].data_ptr(), out["iters"].data_ptr(), out["T"].data_ptr())
    _check(lib().stap_probe(plan.handle, ctypes.c_void_p(x.data_ptr()), H, W, ctypes.c_void_p(pix_t.data_ptr()),
                            npix, ctypes.byref(po), _stream_handle(stream)))
    out["_keep"] = pix_t
    return out


def _tile_array(tiles):
    arr = (StapTile * len(tiles))()
    for i, (plan, x, T, D) in enumerate(tiles):
        H, W = _check_frame(plan, x)
        arr[i] = StapTile(plan.handle.value, x.data_ptr(), H, W, T.data_ptr(),
                          D.data_ptr() if D is not None else None)
    return arr


def run_batch(tiles, stream=None):
    """tiles: list of (plan, x, T, D) with torch tensors; one-shot batched run
    (creates, launches, synchronises and frees a Batch)."""
    _check(lib().stap_run_batch(_tile_array(tiles), len(tiles), _stream_handle(stream)))


def lrstap_probe(plan: Plan, x, pix, r: int = -1, max_iter: int = 0, tol: float = 0.0, stream=None) -> dict:
    """stap_lrstap_probe: the unstructured low-rank STAP baseline on pixels
    pix [(r, c), ...] of a device frame.  Returns T [npix], U [npix, pq, r]
    (complex64, columns by decreasing eigenvalue), lam [npix, r] and iters."""
    import torch
    H, W = _check_frame(plan, x)
    dev = x.device
    if isinstance(pix, torch.Tensor):
        if pix.dtype != torch.int32 or pix.device != dev:
            raise ValueError("pix must be an int32 tensor on the frame's device")
        pix_t = pix.reshape(-1, 2).contiguous()
    else:
        pix_t = torch.as_tensor(np.asarray(pix, dtype=np.int32).reshape(-1, 2), device=dev).contiguous()
    npix = int(pix_t.shape[0])
    rr = plan.r_a * plan.r_b if r < 0 else int(r)
    pq = plan.p * plan.q
    T = torch.zeros(npix, dtype=torch.float32, device=dev)
    U = torch.zeros((npix, pq, max(rr, 0)), dtype=torch.complex64, device=dev)
    lam = torch.zeros((npix, max(rr, 0)), dtype=torch.float32, device=dev)
    iters = torch.zeros(npix, dtype=torch.int32, device=dev)
    cfg = StapLrstapConfig(int(r), int(max_iter), float(tol))
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t.numel() else None  # noqa: E731
    _check(lib().stap_lrstap_probe(plan.handle, ctypes.byref(cfg), ctypes.c_void_p(x.data_ptr()), H, W,
                                   ptr(pix_t), npix, ptr(T), ptr(U), ptr(lam), ptr(iters), _stream_handle(stream)))
    return dict(T=T, U=U, lam=lam, iters=iters, _keep=pix_t)


def sinr_loss(filter: str, a_grid, b_grid, UA_true, lamA_true, UB_true, lamB_true, sigma2: float = 1.0,
              tau2: float = 1.0, UA=None, UB=None, U=None, stream=None):
    """stap_sinr_loss: SINR loss [npix, na, nb] (float32) of per-pixel
    filters ('kron' / 'classical' from UA [npix, p, r_a] and UB [npix, q, r_b],
    'lrstap' from U [npix, pq, r]; complex64 device tensors) for steerings
    a (x) b over a_grid [na, p] x b_grid [nb, q], against the covariance
    tau2 A (x) B + sigma2 I given by orthonormal bases and eigenvalues."""
    import torch
    dev = (U if filter == "lrstap" else UA).device
    c64 = lambda a: torch.as_tensor(np.asarray(a, dtype=np.complex64), device=dev).contiguous()  # noqa: E731
    f64 = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device=dev).contiguous()  # noqa: E731
    ag, bg = c64(a_grid), c64(b_grid)
    uat, ubt, lat, lbt = c64(UA_true), c64(UB_true), f64(lamA_true), f64(lamB_true)
    p, ra = int(uat.shape[0]), int(uat.shape[1])
    q, rb = int(ubt.shape[0]), int(ubt.shape[1])
    na, nb = int(ag.shape[0]), int(bg.shape[0])
    if filter == "lrstap":
        U = U.contiguous()
        npix, r_a, r_b, r = int(U.shape[0]), 0, 0, int(U.shape[2])
    else:
        UA, UB = UA.contiguous(), UB.contiguous()
        npix, r_a, r_b, r = int(UA.shape[0]), int(UA.shape[2]), int(UB.shape[2]), 0
    loss = torch.zeros((npix, na, nb), dtype=torch.float32, device=dev)
    ptr = lambda t: t.data_ptr() if (t is not None and t.numel()) else None  # noqa: E731
    cov = StapTrueCov(p, q, ra, rb, ptr(uat), ptr(lat), ptr(ubt), ptr(lbt), float(sigma2), float(tau2))
    fs = StapFilterSet(SINR_FILTERS[filter], npix, r_a, r_b, r, ptr(UA), ptr(UB), ptr(U))
    _check(lib().stap_sinr_loss(ctypes.byref(cov), ctypes.byref(fs), ctypes.c_void_p(ptr(ag)), na,
                                ctypes.c_void_p(ptr(bg)), nb, ctypes.c_void_p(ptr(loss)), _stream_handle(stream)))
    loss._keep = (ag, bg, uat, ubt, lat, lbt)
    return loss


class Batch:
    """Reusable batch of uneven tiles captured in one HIP graph (see
    stap_batch_create).  Keeps references to the tiles' tensors."""

    def __init__(self, tiles, pix_per_item: int = 0):
        self._tiles = list(tiles)
        self._arr = _tile_array(self._tiles)
        h = ctypes.c_void_p()
        _check(lib().stap_batch_create(self._arr, len(self._tiles), pix_per_item, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().stap_batch_launch(self._h, _stream_handle(stream)))

    def tune(self, stream=None):
        ppb, mult, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().stap_batch_tune(self._h, _stream_handle(stream), ctypes.byref(ppb), ctypes.byref(mult),
                                     ctypes.byref(ms)))
        return dict(pix_per_item=ppb.value, grid_mult=mult.value, ms=ms.value)

    def info(self):
        px, cl, ppb, mult = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().stap_batch_info(self._h, ctypes.byref(px), ctypes.byref(cl), ctypes.byref(ppb),
                                     ctypes.byref(mult)))
        per = []
        for i in range(cl.value):
            v = [ctypes.c_int32() for _ in range(6)]
            _check(lib().stap_batch_class_info(self._h, i, *[ctypes.byref(x) for x in v]))
            per.append(dict(zip(("p", "q", "rb_bound", "precision", "pix_per_item", "grid_mult"), (x.value for x in v))))
        return dict(pixels=px.value, classes=cl.value, pix_per_item=ppb.value, grid_mult=mult.value, per_class=per)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.stap_batch_destroy(h)
            self._h = None


class Server:
    """Continuous-batching server (see stap_server_create).  Frames are host
    numpy/torch-CPU complex64 arrays [p, H, W, q] (pinned torch tensors give
    asynchronous copies) or device torch tensors."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 16, step_pixels: int = 0):
        h = ctypes.c_void_p()
        _check(lib().stap_server_create(int(hbm_budget_bytes), int(max_inflight), int(step_pixels),
                                        ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, plan: Plan, x, with_detections: bool = True) -> int:
        import torch
        if isinstance(x, np.ndarray):
            x = torch.from_numpy(np.ascontiguousarray(x))
        if x.dtype != torch.complex64 or x.dim() != 4 or x.shape[0] != plan.p or x.shape[3] != plan.q:
            raise ValueError("x must be complex64 [p, H, W, q]")
        x = x.contiguous()
        H, W = int(x.shape[1]), int(x.shape[2])
        T = torch.empty((H, W), dtype=torch.float32, pin_memory=True)
        D = torch.empty((H, W), dtype=torch.uint8, pin_memory=True) if with_detections else None
        t = ctypes.c_uint64()
        # a device frame is read only after the work torch has enqueued for it
        stream = _stream_handle(None) if x.is_cuda else None
        _check(lib().stap_server_submit(self._h, plan.handle, ctypes.c_void_p(x.data_ptr()), H, W, int(x.is_cuda),
                                        ctypes.c_void_p(T.data_ptr()),
                                        ctypes.c_void_p(D.data_ptr()) if D is not None else None, stream,
                                        ctypes.byref(t)))
        self._keep[t.value] = (plan, x, T, D)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        lat = ctypes.c_double()
        try:
            _check(lib().stap_server_wait(self._h, ticket, timeout_ms, ctypes.byref(lat)))
        except StapError as e:
            if e.status != 5:
                self._keep.pop(ticket, None)
            raise
        plan, x, T, D = self._keep.pop(ticket)
        return T, D, lat.value

    def stats(self):
        p50, p99, pps, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().stap_server_stats(self._h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(pps),
                                       ctypes.byref(n)))
        return dict(p50_s=p50.value, p99_s=p99.value, pixels_per_s=pps.value, frames=n.value)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.stap_server_destroy(h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        self.close()


def tune_lookup(p: int, q: int, r_b: int, precision: str = "fp32", arch: Optional[str] = None):
    """The tuning cache's entry for a kernel class (see stap_tune_lookup):
    dict(pix_per_item, grid_mult) or None."""
    ppb, mult, found = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().stap_tune_lookup(arch.encode() if arch else None, p, q, r_b, PRECISIONS[precision],
                                  ctypes.byref(ppb), ctypes.byref(mult), ctypes.byref(found)))
    return dict(pix_per_item=ppb.value, grid_mult=mult.value) if found.value else None


def tune_record(p: int, q: int, r_b: int, pix_per_item: int, grid_mult: int, precision: str = "fp32",
                ms: float = 0.0, arch: Optional[str] = None):
    """Records a tuning-cache entry (and rewrites KSTAP_TUNE_CACHE if set)."""
    _check(lib().stap_tune_record(arch.encode() if arch else None, p, q, r_b, PRECISIONS[precision],
                                  pix_per_item, grid_mult, ms))


def version() -> str:
    return lib().stap_version().decode()


def exported_symbols() -> list:
    """Names of the functions declared in include/kstap.h."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "kstap.h")
    txt = open(hdr).read()
    return sorted(set(re.findall(r"^\s*(?:stap_status|const char\*)\s+(stap_\w+)\s*\(", txt, re.M)))
