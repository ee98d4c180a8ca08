"""ctypes binding of librankest (include/rankest.h): argument marshalling only.

Tensors must live on the GPU; every computation runs in the HIP library.  When
the library has not been built, every call raises ``RankEstError`` — there is
no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import threading
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librankest.so")

RE_OK, RE_ERR_INVALID_ARG, RE_ERR_UNSUPPORTED, RE_ERR_NO_MEMORY = 0, -1, -2, -3
RE_ERR_HIP, RE_ERR_NONFINITE, RE_ERR_NO_CONVERGENCE = -4, -5, -6
RE_ERR_SCRATCH_LIMIT = -7
NOALLOC_SCRATCH_BYTES = 16 << 20  # RE_NOALLOC_SCRATCH_BYTES
RE_F64, RE_F32 = 0, 1
RE_GAUSSIAN, RE_SRHT = 0, 1
PREC = {"native": 0, "bf16": 1, "fp16": 2, "auto": 3}
RE_HRTT = 2
RE_SRCT = 3
KIND = {"gaussian": RE_GAUSSIAN, "srht": RE_SRHT, "hrtt": RE_HRTT, "srct": RE_SRCT}
FLAG_NOT_CONVERGED, FLAG_ZERO, FLAG_PREC_FALLBACK, FLAG_USED_BF16, FLAG_USED_FP16 = 1, 2, 4, 8, 16
FLAG_COLUMNS_DROPPED = 32
FLAG_PREC_BELOW_FLOOR = 64
FLAG_SVD_RELAUNCHED = 128
MAX_ADAPTIVE_K = 5120  # RE_MAX_ADAPTIVE_K
FMT = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
FMT_DTYPE = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16, 3: torch.float16}
STAGES = ("x_draw", "ax", "y_draw", "yb", "svd", "rank")
NUM_STAGES = len(STAGES)


class RankEstError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        msg = _status_text(status)
        super().__init__(f"{where}: {msg} (status {status})" if where else f"{msg} (status {status})")
        self.status = status


class ReSketch(C.Structure):
    _fields_ = [("x_kind", C.c_int32), ("y_kind", C.c_int32), ("k", C.c_int32), ("l", C.c_int32),
                ("prec", C.c_int32)]


class ReAdaptive(C.Structure):
    _fields_ = [("k0", C.c_int32), ("k_max", C.c_int32), ("l_ratio", C.c_double), ("mlp", C.c_void_p),
                ("delta", C.c_double)]


class ReGapSearch(C.Structure):
    _fields_ = [("k0", C.c_int32), ("dk", C.c_int32), ("k_max", C.c_int32), ("y_kind", C.c_int32),
                ("l_ratio", C.c_double), ("gamma", C.c_double), ("floor", C.c_double)]


MLP_INPUTS, MLP_PARAMS = 35, 6529


class ReBlock(C.Structure):
    _fields_ = [("A", C.c_void_p), ("m", C.c_int64), ("n", C.c_int64), ("lda", C.c_int64)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load librankest.so; raises RankEstError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RankEstError(RE_ERR_HIP, f"HIP library missing at {LIB_PATH}; build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "re_create": ([C.POINTER(vp), vp], i32),
            "re_destroy": ([vp], i32),
            "re_set_stream": ([vp, vp], i32),
            "re_workspace_bytes": ([vp, C.POINTER(C.c_size_t)], i32),
            "re_set_profiling": ([vp, i32], i32),
            "re_set_limits": ([vp, i64, i64], i32),
            "re_last_stage_ms": ([vp, vp], i32),
            "re_rank_estimate": ([vp, vp, i32, i64, i64, i64, dbl, C.POINTER(ReSketch), u64, C.POINTER(i32), vp,
                                  C.POINTER(i32), C.POINTER(C.c_uint32)], i32),
            "re_rank_estimate_qr": ([vp, vp, i32, i64, i64, i64, dbl, C.POINTER(ReSketch), u64, C.POINTER(i32), vp,
                                     C.POINTER(i32), C.POINTER(C.c_uint32)], i32),
            "re_rank_estimate_batched": ([vp, vp, i32, i32, dbl, C.POINTER(ReSketch), u64, vp, vp, vp], i32),
            "re_rank_adaptive": ([vp, vp, i32, i64, i64, i64, dbl, C.POINTER(ReAdaptive), u64, C.POINTER(i32), vp,
                                  C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                  C.POINTER(C.c_uint32)], i32),
            "re_rank_adaptive_y": ([vp, vp, i32, i64, i64, i64, dbl, C.POINTER(ReAdaptive), i32, u64, C.POINTER(i32),
                                    vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                    C.POINTER(C.c_uint32)], i32),
            "re_rangefinder": ([vp, vp, i32, i64, i64, i64, dbl, i32, C.POINTER(ReAdaptive), dbl, u64, vp, i64, vp,
                                i64, C.POINTER(i32), C.POINTER(i32), vp, C.POINTER(i32), C.POINTER(C.c_uint32)], i32),
            "re_rank_gap": ([vp, vp, i32, i64, i64, i64, C.POINTER(ReGapSearch), u64, C.POINTER(i32),
                             C.POINTER(dbl), C.POINTER(i32), C.POINTER(dbl), vp, C.POINTER(i32), C.POINTER(i32),
                             C.POINTER(i32), vp, i32, C.POINTER(C.c_uint32)], i32),
            "re_rangefinder_stage_ms": ([vp, vp], i32),
            "re_thin_qr": ([vp, vp, i32, i64, i64, i64, vp, i64, C.POINTER(i32), C.POINTER(C.c_uint32)], i32),
            "re_project": ([vp, vp, i64, i64, vp, i32, i64, i64, i64, vp, i64], i32),
            "re_mlp_forward": ([vp, vp, vp, i64, vp], i32),
            "re_mlp_loss_grad": ([vp, vp, vp, vp, i64, vp, vp], i32),
            "re_mlp_adam": ([vp, vp, vp, vp, vp, i64, i32, dbl, dbl, dbl, dbl], i32),
            "re_philox": ([vp, vp, u64, i64, vp], i32),
            "re_gauss_fill": ([vp, i32, i64, i64, u64, i32, i32, vp], i32),
            "re_srht_signs": ([vp, i64, u64, i32, vp], i32),
            "re_srht_select": ([vp, i64, i64, u64, i32, vp], i32),
            "re_sketch_x": ([vp, vp, i32, i64, i64, i64, C.POINTER(ReSketch), u64, vp], i32),
            "re_sketch_y": ([vp, vp, i32, i64, i64, C.POINTER(ReSketch), u64, vp], i32),
            "re_sketch_y_rows": ([i64], i64),
            "re_singular_values": ([vp, vp, i64, i64, dbl, vp], i32),
            "re_singular_values_noalloc": ([vp, vp, i64, i64, dbl, vp], i32),
            "re_singular_values_noalloc_fits": ([i64, i64], i32),
            "re_rank_count": ([vp, vp, i64, i32, dbl, vp], i32),
            "re_r1_from_k": ([i32], i32),
            "re_gap_rank": ([vp, i32, i32, C.POINTER(i32), C.POINTER(dbl)], i32),
            "re_status_string": ([i32], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        return _lib


def _status_text(status: int) -> str:
    try:
        return lib().re_status_string(status).decode()
    except Exception:
        return "librankest status"


def _check(st: int, where: str):
    if st != RE_OK:
        raise RankEstError(st, where)


class Handle:
    """One library handle bound to a device; follows torch's current stream."""

    def __init__(self, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index)
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().re_create(C.byref(self._h), C.c_void_p(torch.cuda.current_stream().cuda_stream)), "re_create")
        self._stream = torch.cuda.current_stream(self.device).cuda_stream
        _live.add(self)

    def bind(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            _check(lib().re_set_stream(self._h, C.c_void_p(s)), "re_set_stream")
            self._stream = s
        return self._h

    def workspace_bytes(self) -> int:
        n = C.c_size_t(0)
        _check(lib().re_workspace_bytes(self._h, C.byref(n)), "re_workspace_bytes")
        return n.value

    def set_profiling(self, enable: bool = True):
        _check(lib().re_set_profiling(self._h, int(bool(enable))), "re_set_profiling")

    def set_limits(self, max_workspace_bytes: int = 0, barrier_polls: int = 0):
        """Cap on each of the handle's workspaces (0: none) and the polls of the
        small SVD's grid barriers before RE_ERR_NO_CONVERGENCE (0: default,
        negative: at the first poll)."""
        _check(lib().re_set_limits(self._h, int(max_workspace_bytes), int(barrier_polls)), "re_set_limits")

    def last_stage_ms(self) -> dict:
        """Per-stage durations (ms) of the last rank_estimate on this handle (HIP events)."""
        ms = np.zeros(NUM_STAGES, dtype=np.float64)
        _check(lib().re_last_stage_ms(self._h, ms.ctypes.data_as(C.c_void_p)), "re_last_stage_ms")
        return dict(zip(STAGES, ms.tolist()))

    def close(self):
        if self._h:
            lib().re_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        # At interpreter shutdown the HIP runtime (and a profiler attached to
        # it) may already be gone; handles still open then were released by
        # _close_all at exit, so nothing is left to do here.  Late in the
        # shutdown even module globals such as `sys` may already be None.
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass


_handles: dict = {}
_live = weakref.WeakSet()


def _close_all():
    """Release every open handle while the HIP runtime is still alive: Python's
    exit hooks run before the runtime's own teardown, whereas a handle left to
    the garbage collector may be destroyed after it."""
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass
    _handles.clear()


atexit.register(_close_all)
close_all_handles = _close_all


def default_handle(device=None) -> Handle:
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    h = _handles.get(dev)
    if h is None:
        h = _handles[dev] = Handle(dev)
    return h


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _need_cuda(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return RE_F64
    if t.dtype == torch.float32:
        return RE_F32
    raise ValueError("A must be float32 or float64")


def make_sketch(k: int, l: int = 0, x: str = "gaussian", y: str = "gaussian", precision: str = "native") -> ReSketch:
    return ReSketch(KIND[x], KIND[y], int(k), int(l), PREC[precision])


def _check_matrix(A: torch.Tensor):
    _need_cuda(A, "A")
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D tensor with unit column stride")


def rank_estimate(A: torch.Tensor, eps: float, *, k: int, l: int = 0, x: str = "gaussian", y: str = "gaussian",
                  precision: str = "native", seed: int = 0, handle: Handle | None = None):
    """Algorithm 1 on one matrix.  Returns (r, sigma[k] (numpy float64), info dict)."""
    _check_matrix(A)
    h = handle or default_handle(A.device)
    m, n = A.shape
    sk = make_sketch(k, l, x, y, precision)
    r = C.c_int32(0)
    r1 = C.c_int32(0)
    fl = C.c_uint32(0)
    sigma = np.zeros(int(k), dtype=np.float64)
    st = lib().re_rank_estimate(h.bind(), _ptr(A), _dtype_code(A), m, n, A.stride(0), float(eps), C.byref(sk),
                                int(seed) % 2**64, C.byref(r), sigma.ctypes.data_as(C.c_void_p), C.byref(r1),
                                C.byref(fl))
    _check(st, "re_rank_estimate")
    return r.value, sigma, {"r1": r1.value, "flags": fl.value, "k": int(k), "l": int(l) if l else 2 * int(k)}


def rank_estimate_qr(A: torch.Tensor, eps: float, *, k: int, l: int = 0, x: str = "gaussian", y: str = "gaussian",
                     seed: int = 0, handle: Handle | None = None):
    """Algorithm 1 with step 7 by the diagonal of R in Y A X = Q R (Sec. 5).
    Returns (r, d[k] (sorted |R_jj| / sqrt(k l), numpy float64), info dict)."""
    _check_matrix(A)
    h = handle or default_handle(A.device)
    m, n = A.shape
    sk = make_sketch(k, l, x, y, "native")
    r = C.c_int32(0)
    r1 = C.c_int32(0)
    fl = C.c_uint32(0)
    d = np.zeros(int(k), dtype=np.float64)
    st = lib().re_rank_estimate_qr(h.bind(), _ptr(A), _dtype_code(A), m, n, A.stride(0), float(eps), C.byref(sk),
                                   int(seed) % 2**64, C.byref(r), d.ctypes.data_as(C.c_void_p), C.byref(r1),
                                   C.byref(fl))
    _check(st, "re_rank_estimate_qr")
    return r.value, d, {"r1": r1.value, "flags": fl.value, "k": int(k), "l": int(l) if l else 2 * int(k)}


def rank_adaptive(A: torch.Tensor, eps: float, *, k0: int = 32, k_max: int = 0, l_ratio: float = 1.5,
                  mlp: torch.Tensor | None = None, delta: float = 0.0, seed: int = 0, y: str = "gaussian",
                  handle: Handle | None = None):
    """Rank estimate with an adaptive sketch width (FP32 A, Gaussian X; Y
    Gaussian or, with y="srht", the SRHT grown from its stored transform):
    doubling from k0, or the network's proposal after the pilot when `mlp`
    (device float32 parameter vector) is given.  Returns (r, sigma, info) with
    info = {k, l, rounds, k_proposed, flags}."""
    _check_matrix(A)
    if mlp is not None:
        _need_cuda(mlp, "mlp")
        if mlp.dtype != torch.float32 or mlp.numel() != MLP_PARAMS or not mlp.is_contiguous():
            raise ValueError(f"mlp must be a contiguous float32 tensor of {MLP_PARAMS} values")
    h = handle or default_handle(A.device)
    m, n = A.shape
    ad = ReAdaptive(int(k0), int(k_max), float(l_ratio), mlp.data_ptr() if mlp is not None else None, float(delta))
    kcap = min(m, n, MAX_ADAPTIVE_K) if k_max <= 0 else min(m, n, k_max, MAX_ADAPTIVE_K)
    sigma = np.zeros(kcap, dtype=np.float64)
    r, kk, ll, rounds, kp = (C.c_int32(0) for _ in range(5))
    fl = C.c_uint32(0)
    if y == "gaussian":
        st = lib().re_rank_adaptive(h.bind(), _ptr(A), _dtype_code(A), m, n, A.stride(0), float(eps), C.byref(ad),
                                    int(seed) % 2**64, C.byref(r), sigma.ctypes.data_as(C.c_void_p), C.byref(kk),
                                    C.byref(ll), C.byref(rounds), C.byref(kp), C.byref(fl))
    else:
        st = lib().re_rank_adaptive_y(h.bind(), _ptr(A), _dtype_code(A), m, n, A.stride(0), float(eps),
                                      C.byref(ad), KIND[y], int(seed) % 2**64, C.byref(r),
                                      sigma.ctypes.data_as(C.c_void_p), C.byref(kk), C.byref(ll), C.byref(rounds),
                                      C.byref(kp), C.byref(fl))
    _check(st, "re_rank_adaptive")
    return r.value, sigma[:kk.value], {"k": kk.value, "l": ll.value, "rounds": rounds.value,
                                       "k_proposed": kp.value, "flags": fl.value}


def rank_gap(A: torch.Tensor, *, k0: int = 110, dk: int = 100, k_max: int = 0, l_ratio: float = 1.5,
             gamma: float = 100.0, floor: float | None = None, y: str = "gaussian", seed: int = 0,
             spectra: int = 64, handle: Handle | None = None):
    """Rank without a tolerance (re_rank_gap): the search of Sec. 6.1 on an
    FP32 or FP64 A with a Gaussian X grown by dk columns per round and a
    Gaussian or SRHT Y.  floor defaults to 1e-13 (FP64 A) or 1e-5 (FP32 A).
    Returns (r, sigma, info) with r the deepest stable gap and info = {ratio,
    argmax, argmax_ratio, k, l, rounds, flags, spectra (one array per round,
    the first `spectra` rounds)}."""
    _check_matrix(A)
    h = handle or default_handle(A.device)
    m, n = A.shape
    if floor is None:
        floor = 1e-13 if A.dtype == torch.float64 else 1e-5
    gs = ReGapSearch(int(k0), int(dk), int(k_max), KIND[y], float(l_ratio), float(gamma), float(floor))
    kcap = min(m, n, MAX_ADAPTIVE_K) if k_max <= 0 else min(m, n, k_max, MAX_ADAPTIVE_K)
    sigma = np.zeros(kcap, dtype=np.float64)
    spec = np.zeros((max(int(spectra), 0), kcap), dtype=np.float64)
    r, a, kk, ll, rounds = (C.c_int32(0) for _ in range(5))
    q, qa = C.c_double(0.0), C.c_double(0.0)
    fl = C.c_uint32(0)
    st = lib().re_rank_gap(h.bind(), _ptr(A), _dtype_code(A), m, n, A.stride(0), C.byref(gs), int(seed) % 2**64,
                           C.byref(r), C.byref(q), C.byref(a), C.byref(qa), sigma.ctypes.data_as(C.c_void_p),
                           C.byref(kk), C.byref(ll), C.byref(rounds),
                           spec.ctypes.data_as(C.c_void_p) if spec.size else None, spec.shape[0], C.byref(fl))
    _check(st, "re_rank_gap")
    widths = []
    k = min(int(k0), kcap)
    for _ in range(min(rounds.value, spec.shape[0])):
        widths.append(k)
        k = min(k + int(dk), kcap)
    return r.value, sigma[:kk.value], {"ratio": q.value, "argmax": a.value, "argmax_ratio": qa.value, "k": kk.value,
                                       "l": ll.value, "rounds": rounds.value, "flags": fl.value,
                                       "spectra": [spec[j, :w].copy() for j, w in enumerate(widths)]}


def rangefinder(A: torch.Tensor, eps: float, p: int = 10, *, k0: int = 32, k_max: int = 0, l_ratio: float = 2.0,
                norm_a: float = 0.0, seed: int = 0, Q: torch.Tensor | None = None, B: torch.Tensor | None = None,
                handle: Handle | None = None):
    """Rank estimation followed by the randomized rangefinder (FP32 A): the
    fixed-precision factorisation A ~ Q B of rank w.  Q (m x k_max capacity)
    and B (k_max x n capacity) are FP64 device tensors, allocated here unless
    given.  Returns (Q[:, :w], B[:w], info) with info = {r, w, k, sigma, flags}."""
    _check_matrix(A)
    h = handle or default_handle(A.device)
    m, n = A.shape
    kcap = min(m, n, MAX_ADAPTIVE_K) if k_max <= 0 else min(m, n, k_max, MAX_ADAPTIVE_K)
    if Q is None:
        Q = torch.empty(m, kcap, dtype=torch.float64, device=A.device)
    if B is None:
        B = torch.empty(kcap, n, dtype=torch.float64, device=A.device)
    for t, name in ((Q, "Q"), (B, "B")):
        _need_cuda(t, name)
        if t.dtype != torch.float64 or t.stride(1) != 1:
            raise ValueError(f"{name} must be a float64 tensor with unit column stride")
    if Q.shape[0] < m or Q.shape[1] < kcap or B.shape[0] < kcap or B.shape[1] < n:
        raise ValueError("Q must hold m x k_max and B k_max x n values")
    ad = ReAdaptive(int(k0), int(k_max), float(l_ratio), None, 0.0)
    sigma = np.zeros(kcap, dtype=np.float64)
    r, w, kk = (C.c_int32(0) for _ in range(3))
    fl = C.c_uint32(0)
    st = lib().re_rangefinder(h.bind(), _ptr(A), _dtype_code(A), m, n, A.stride(0), float(eps), int(p), C.byref(ad),
                              float(norm_a), int(seed) % 2**64, _ptr(Q), Q.stride(0), _ptr(B), B.stride(0),
                              C.byref(r), C.byref(w), sigma.ctypes.data_as(C.c_void_p), C.byref(kk), C.byref(fl))
    _check(st, "re_rangefinder")
    wv = w.value
    return Q[:m, :wv], B[:wv, :n], {"r": r.value, "w": wv, "k": kk.value, "sigma": sigma[:kk.value],
                                    "flags": fl.value}


def thin_qr(W: torch.Tensor, handle: Handle | None = None):
    """Orthonormal basis of the columns of W (m x w, FP32 or FP64, on the GPU)
    by the library's shifted CholeskyQR3.  Returns (Q[:, :w_kept], flags)."""
    _check_matrix(W)
    m, w = W.shape
    Q = torch.empty(m, w, dtype=torch.float64, device=W.device)
    h = handle or default_handle(W.device)
    we = C.c_int32(0)
    fl = C.c_uint32(0)
    _check(lib().re_thin_qr(h.bind(), _ptr(W), _dtype_code(W), m, w, W.stride(0), _ptr(Q), Q.stride(0),
                            C.byref(we), C.byref(fl)), "re_thin_qr")
    return Q[:, :we.value], fl.value


def project(Q: torch.Tensor, A: torch.Tensor, handle: Handle | None = None) -> torch.Tensor:
    """B = Q^T A for FP64 Q (m x w) and FP32 A (m x n) on the GPU; B is FP64."""
    _check_matrix(A)
    _need_cuda(Q, "Q")
    if Q.dtype != torch.float64 or Q.stride(1) != 1 or Q.shape[0] != A.shape[0]:
        raise ValueError("Q must be a float64 m x w tensor with unit column stride")
    m, n = A.shape
    w = Q.shape[1]
    B = torch.empty(w, n, dtype=torch.float64, device=A.device)
    h = handle or default_handle(A.device)
    _check(lib().re_project(h.bind(), _ptr(Q), Q.stride(0), w, _ptr(A), _dtype_code(A), m, n, A.stride(0), _ptr(B),
                            B.stride(0)), "re_project")
    return B


def rangefinder_stage_ms(handle: Handle | None = None) -> list[float]:
    """Stage times of the last profiled rangefinder call: estimation, thin QR, Q^T A."""
    h = handle or default_handle()
    ms = np.zeros(3, dtype=np.float64)
    _check(lib().re_rangefinder_stage_ms(h.bind(), ms.ctypes.data_as(C.c_void_p)), "re_rangefinder_stage_ms")
    return ms.tolist()


def mlp_forward(params: torch.Tensor, x: torch.Tensor, handle: Handle | None = None) -> torch.Tensor:
    """Network outputs for a batch of feature rows (device float32)."""
    _need_cuda(params, "params")
    _need_cuda(x, "x")
    x = x.contiguous()
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    h = handle or default_handle(x.device)
    _check(lib().re_mlp_forward(h.bind(), _ptr(params), _ptr(x), x.shape[0], _ptr(y)), "re_mlp_forward")
    return y


def mlp_loss_grad(params: torch.Tensor, x: torch.Tensor, t: torch.Tensor, handle: Handle | None = None):
    """(gradient of the mean squared error, loss) on device, float32."""
    x = x.contiguous()
    t = t.contiguous()
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    h = handle or default_handle(x.device)
    _check(lib().re_mlp_loss_grad(h.bind(), _ptr(params), _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss)),
           "re_mlp_loss_grad")
    return g, loss


def mlp_adam(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
             beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, handle: Handle | None = None):
    """One Adam step in place on device float32 tensors."""
    h = handle or default_handle(params.device)
    _check(lib().re_mlp_adam(h.bind(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), int(step),
                             float(lr), float(beta1), float(beta2), float(eps)), "re_mlp_adam")


def make_blocks(blocks) -> "C.Array[ReBlock]":
    """Descriptor table of a batched call from FP32 GPU matrices (row-major views
    with unit column stride).  The table holds raw pointers: keep the tensors
    alive while it is in use."""
    arr = (ReBlock * len(blocks))()
    for i, A in enumerate(blocks):
        _check_matrix(A)
        if A.dtype != torch.float32:
            raise ValueError("batched blocks must be float32")
        arr[i].A = A.data_ptr()
        arr[i].m, arr[i].n = A.shape
        arr[i].lda = A.stride(0)
    return arr


def rank_estimate_batched(blocks, eps: float, *, k: int, l: int = 0, seed: int = 0, handle: Handle | None = None):
    """Algorithm 1 on many FP32 blocks in one graph launch (Gaussian X and Y).

    ``blocks`` is a list of GPU tensors or a table from ``make_blocks``.
    Returns (r int32[nb], sigma float64[nb, k], flags uint32[nb])."""
    table = blocks if isinstance(blocks, C.Array) else make_blocks(blocks)
    nb = len(table)
    if nb == 0:
        return np.zeros(0, np.int32), np.zeros((0, int(k))), np.zeros(0, np.uint32)
    dev = torch.device("cuda", torch.cuda.current_device()) if handle is None else handle.device
    h = handle or default_handle(dev)
    sk = make_sketch(k, l, "gaussian", "gaussian", "native")
    r = np.zeros(nb, dtype=np.int32)
    sigma = np.zeros((nb, int(k)), dtype=np.float64)
    fl = np.zeros(nb, dtype=np.uint32)
    st = lib().re_rank_estimate_batched(h.bind(), C.cast(table, C.c_void_p), nb, RE_F32, float(eps), C.byref(sk),
                                        int(seed) % 2**64, r.ctypes.data_as(C.c_void_p),
                                        sigma.ctypes.data_as(C.c_void_p), fl.ctypes.data_as(C.c_void_p))
    _check(st, "re_rank_estimate_batched")
    return r, sigma, fl


# --- stage entry points ------------------------------------------------------------------------

def philox(ctr: torch.Tensor, seed: int, handle: Handle | None = None) -> torch.Tensor:
    """ctr: int64 CUDA tensor (count, 4) holding the uint64 counter bits."""
    _need_cuda(ctr, "ctr")
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    h = handle or default_handle(ctr.device)
    _check(lib().re_philox(h.bind(), _ptr(ctr), int(seed) % 2**64, ctr.shape[0], _ptr(out)), "re_philox")
    return out


def gauss_fill(fmt: str, rows: int, cols: int, seed: int, stream_id: int, swap_ab: bool = False,
               device="cuda", handle: Handle | None = None) -> torch.Tensor:
    code = FMT[fmt]
    out = torch.empty(rows, cols, dtype=FMT_DTYPE[code], device=device)
    h = handle or default_handle(out.device)
    _check(lib().re_gauss_fill(h.bind(), code, rows, cols, int(seed) % 2**64, stream_id, int(swap_ab), _ptr(out)),
           "re_gauss_fill")
    return out


def srht_signs(npad: int, seed: int, stream_id: int, device="cuda", handle: Handle | None = None) -> torch.Tensor:
    """Packed sign bits (int32 view of the uint32 words); bit set = -1."""
    out = torch.zeros((npad + 31) // 32, dtype=torch.int32, device=device)
    h = handle or default_handle(out.device)
    _check(lib().re_srht_signs(h.bind(), npad, int(seed) % 2**64, stream_id, _ptr(out)), "re_srht_signs")
    return out


def srht_select(npad: int, k: int, seed: int, stream_id: int, device="cuda", handle: Handle | None = None):
    out = torch.empty(max(k, 1), dtype=torch.int32, device=device)
    h = handle or default_handle(out.device)
    _check(lib().re_srht_select(h.bind(), npad, k, int(seed) % 2**64, stream_id, _ptr(out)), "re_srht_select")
    return out[:k]


def sketch_x(A: torch.Tensor, *, k: int, l: int = 0, x: str = "gaussian", y: str = "gaussian",
             precision: str = "native", seed: int = 0, handle: Handle | None = None) -> torch.Tensor:
    """B = A X (unscaled), m x k, FP64 for an FP64 A else FP32."""
    _check_matrix(A)
    m, n = A.shape
    B = torch.empty(m, k, dtype=A.dtype, device=A.device)
    sk = make_sketch(k, l, x, y, precision)
    h = handle or default_handle(A.device)
    _check(lib().re_sketch_x(h.bind(), _ptr(A), _dtype_code(A), m, n, A.stride(0), C.byref(sk), int(seed) % 2**64,
                             _ptr(B)), "re_sketch_x")
    return B


def sketch_y(B: torch.Tensor, *, l: int, x: str = "gaussian", y: str = "gaussian", seed: int = 0,
             handle: Handle | None = None) -> torch.Tensor:
    """C = Y B (unscaled), l x k FP64.  B is copied into a scratch buffer first."""
    _need_cuda(B, "B")
    m, k = B.shape
    rows = lib().re_sketch_y_rows(m)
    scratch = torch.zeros(max(rows, m), k, dtype=B.dtype, device=B.device)
    scratch[:m].copy_(B)
    Cm = torch.empty(l, k, dtype=torch.float64, device=B.device)
    sk = make_sketch(k, l, x, y, "native")
    h = handle or default_handle(B.device)
    _check(lib().re_sketch_y(h.bind(), _ptr(scratch), _dtype_code(B), m, k, C.byref(sk), int(seed) % 2**64, _ptr(Cm)),
           "re_sketch_y")
    return Cm


def singular_values(Cm: torch.Tensor, scale: float = 1.0, handle: Handle | None = None) -> torch.Tensor:
    _need_cuda(Cm, "C")
    Cm = Cm.to(torch.float64).contiguous()
    l, k = Cm.shape
    sigma = torch.empty(k, dtype=torch.float64, device=Cm.device)
    h = handle or default_handle(Cm.device)
    _check(lib().re_singular_values(h.bind(), _ptr(Cm), l, k, float(scale), _ptr(sigma)), "re_singular_values")
    return sigma


def singular_values_noalloc(Cm: torch.Tensor, sigma: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
    """re_singular_values_noalloc on torch's current stream: the singular values
    of the l x k FP64 device matrix Cm into the caller's k-element FP64 device
    tensor sigma, with no device allocation inside the library (fixed per-GPU
    scratch; overlapping calls on one GPU race).  Does not synchronise."""
    _need_cuda(Cm, "C")
    _need_cuda(sigma, "sigma")
    if Cm.dtype != torch.float64 or not Cm.is_contiguous() or Cm.dim() != 2:
        raise ValueError("C must be a contiguous 2-D float64 tensor")
    l, k = Cm.shape
    if sigma.dtype != torch.float64 or not sigma.is_contiguous() or sigma.numel() < k:
        raise ValueError("sigma must be a contiguous float64 tensor of at least k elements")
    with torch.cuda.device(Cm.device):
        st = torch.cuda.current_stream(Cm.device).cuda_stream
        _check(lib().re_singular_values_noalloc(C.c_void_p(st), _ptr(Cm), l, k, float(scale), _ptr(sigma)),
               "re_singular_values_noalloc")
    return sigma


def rank_count(sigma: torch.Tensor, r1: int, eps: float, handle: Handle | None = None):
    _need_cuda(sigma, "sigma")
    sigma = sigma.to(torch.float64).contiguous()
    out = torch.zeros(4, dtype=torch.int32, device=sigma.device)
    h = handle or default_handle(sigma.device)
    _check(lib().re_rank_count(h.bind(), _ptr(sigma), sigma.numel(), int(r1), float(eps), _ptr(out)), "re_rank_count")
    o = out.cpu().tolist()
    return o[0], o[1], o[2]


def gap_rank(sigma, r1: int):
    """Rank without a tolerance from the largest gap of the first r1 estimates
    (host-only).  Returns (r, ratio)."""
    s = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64))
    r = C.c_int32(0)
    q = C.c_double(0.0)
    _check(lib().re_gap_rank(s.ctypes.data_as(C.c_void_p), int(s.size), int(r1), C.byref(r), C.byref(q)),
           "re_gap_rank")
    return r.value, q.value


def r1_from_k(k: int) -> int:
    return lib().re_r1_from_k(int(k))
