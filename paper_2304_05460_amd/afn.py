"""Python binding of libafn (include/afn.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch device
tensors to raw pointers and the current torch stream to a hipStream_t, checks
shapes, and turns non-zero status codes into exceptions.  There is no CPU
fallback: without the built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import pathlib

import torch

_PKG = pathlib.Path(__file__).resolve().parent
LIB_PATH = _PKG / "libafn.so"
_lib = None

AFN_OK, AFN_EINVAL, AFN_ENOMEM, AFN_ENOTSPD, AFN_ENOCONV, AFN_EBREAKDOWN, AFN_ESTAGNATION, \
    AFN_EDEVICE = range(8)
AFN_FP64, AFN_FP32, AFN_BF16 = 0, 1, 2
AFN_METHOD_AFN, AFN_METHOD_NYSTROM, AFN_METHOD_AUTO = 0, 1, 2
AFN_LANDMARKS_AUTO, AFN_LANDMARKS_FPS, AFN_LANDMARKS_UNIFORM = 0, 1, 2
AFN_KERNEL_GAUSSIAN, AFN_KERNEL_MATERN32 = 0, 1
AFN_TUNE_OFF, AFN_TUNE_ON, AFN_TUNE_FORCE = 0, 1, 2
_STATUS_NAMES = ["AFN_OK", "AFN_EINVAL", "AFN_ENOMEM", "AFN_ENOTSPD", "AFN_ENOCONV",
                 "AFN_EBREAKDOWN", "AFN_ESTAGNATION", "AFN_EDEVICE"]


def status_name(status: int) -> str:
    return _STATUS_NAMES[status] if 0 <= status < len(_STATUS_NAMES) else f"status {status}"

EXPORTED = ["kernel_matvec", "kernel_matvec_ex", "kernel_matvec_noalloc", "afn_workspace_size", "afn_setup",
            "afn_apply", "afn_pcg_solve", "afn_pcg_begin", "afn_pcg_step_many", "afn_pcg_query",
            "afn_pcg_end", "afn_get_info", "afn_get_landmarks", "afn_get_fsai", "afn_get_cholesky",
            "afn_footprint_bytes", "afn_tune_config", "afn_tune_report", "afn_destroy", "afn_status_string",
            "afn_last_error", "afn_group_config"]


class AFNError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().afn_last_error().decode(errors="replace")
        name = lib().afn_status_string(status).decode(errors="replace")
        super().__init__(f"{where}: {name}: {msg}")
        self.status = status


class afn_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("k_max", ctypes.c_int32), ("w", ctypes.c_int32),
                ("m", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("method", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("landmarks", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("nrhs_max", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class afn_setup_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32),
                ("w", ctypes.c_int32), ("rank_r", ctypes.c_int32),
                ("rank_k_est", ctypes.c_int64), ("rank_eig_branch", ctypes.c_int32),
                ("rank_eig_count", ctypes.c_int32), ("nnz_g", ctypes.c_int64),
                ("ms_rank", ctypes.c_double), ("ms_fps", ctypes.c_double),
                ("ms_chol", ctypes.c_double), ("ms_knn", ctypes.c_double),
                ("ms_v", ctypes.c_double), ("ms_fsai", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("method", ctypes.c_int32),
                ("landmarks", ctypes.c_int32), ("nu", ctypes.c_double),
                ("kmv_kept_f64", ctypes.c_double), ("kmv_kept_f32", ctypes.c_double),
                ("kmv_far_f64", ctypes.c_double), ("ws_bytes", ctypes.c_int64),
                ("ws_bytes_used", ctypes.c_int64)]


class afn_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("ms_solve", ctypes.c_double), ("ms_matvec", ctypes.c_double),
                ("matvec_launches", ctypes.c_int32), ("outer_iterations", ctypes.c_int32),
                ("fp64_iterations", ctypes.c_int32), ("grouped_units", ctypes.c_int32)]


def lib():
    """Load libafn.so (building it if it was never built); raises if impossible."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(str(LIB_PATH))
        _declare(L)
        _lib = L
    return _lib


_P, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double


def _declare(L):
    L.kernel_matvec.argtypes = [_P, _I64, _I32, _D, _D, _P, _P, _I32, _I64, _I32, _P]
    L.kernel_matvec_ex.argtypes = [_P, _I64, _I32, _D, _D, _P, _P, _I32, _I64, _I32, _I32, _P]
    L.kernel_matvec_noalloc.argtypes = [_P, _I64, _I32, _D, _D, _P, _P, _I32, _I64, _I32, _I32, _P]
    L.afn_setup.argtypes = [_P, _I64, _I32, _D, _D, ctypes.POINTER(afn_params), _P, ctypes.c_size_t,
                            _P, ctypes.POINTER(_P)]
    L.afn_workspace_size.argtypes = [_I64, _I32, ctypes.POINTER(afn_params),
                                     ctypes.POINTER(ctypes.c_size_t)]
    L.afn_pcg_begin.argtypes = [_P, _P, _P, _D, _I32, _P, ctypes.POINTER(_P)]
    L.afn_pcg_step_many.argtypes = [ctypes.POINTER(_P), _I32, _I32, _P]
    L.afn_pcg_query.argtypes = [_P, ctypes.POINTER(_I32), ctypes.POINTER(afn_solve_info)]
    L.afn_pcg_end.argtypes = [_P]
    L.afn_pcg_end.restype = None
    L.afn_group_config.argtypes = [_I32]
    L.afn_group_config.restype = None
    L.afn_tune_config.argtypes = [_I32, _I32, ctypes.c_char_p]
    L.afn_tune_report.argtypes = [ctypes.c_char_p, _I64, ctypes.POINTER(_I64)]
    L.afn_apply.argtypes = [_P, _P, _P, _I32, _I64, _P]
    L.afn_pcg_solve.argtypes = [_P, _P, _P, _I32, _I64, _D, _I32,
                                ctypes.POINTER(afn_solve_info), _P]
    L.afn_get_info.argtypes = [_P, ctypes.POINTER(afn_setup_info)]
    L.afn_get_landmarks.argtypes = [_P, _P, _I64, ctypes.POINTER(_I64)]
    L.afn_get_fsai.argtypes = [_P, _P, _P, _P, _I64, ctypes.POINTER(_I64)]
    L.afn_get_cholesky.argtypes = [_P, _P, _I64]
    L.afn_footprint_bytes.argtypes = [_I64, _I32, ctypes.POINTER(afn_params),
                                      ctypes.POINTER(ctypes.c_size_t)]
    L.afn_destroy.argtypes = [_P]
    L.afn_destroy.restype = None
    L.afn_status_string.argtypes = [ctypes.c_int]
    L.afn_status_string.restype = ctypes.c_char_p
    L.afn_last_error.argtypes = []
    L.afn_last_error.restype = ctypes.c_char_p
    for name in ("kernel_matvec", "kernel_matvec_ex", "kernel_matvec_noalloc", "afn_workspace_size", "afn_setup",
                 "afn_apply", "afn_pcg_solve", "afn_pcg_begin", "afn_pcg_step_many", "afn_pcg_query",
                 "afn_get_info", "afn_get_landmarks", "afn_get_fsai", "afn_get_cholesky", "afn_footprint_bytes",
                 "afn_tune_config", "afn_tune_report"):
        getattr(L, name).restype = ctypes.c_int


def _check(st: int, where: str, ok=(AFN_OK,)):
    if st not in ok:
        raise AFNError(st, where)
    return st


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 CUDA (HIP) tensor")
    return t


def _colmajor(t: torch.Tensor, name: str):
    """(n,) or (n, nrhs) column-major FP64 device tensor -> (ptr, nrhs, ld)."""
    _dev_f64(t, name)
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise ValueError(f"{name} must be contiguous")
        return t.data_ptr(), 1, t.shape[0]
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError(f"{name} must be (n,) or column-major (n, nrhs) (stride(0) == 1)")
    return t.data_ptr(), t.shape[1], max(t.stride(1), t.shape[0])


def empty_colmajor(n: int, nrhs: int, device=None) -> torch.Tensor:
    """A column-major (n, nrhs) float64 device tensor."""
    return torch.empty((nrhs, n), dtype=torch.float64, device=device or "cuda").t()


def kernel_matvec(X: torch.Tensor, l: float, mu: float, v: torch.Tensor,
                  precision: int = AFN_FP64, out: torch.Tensor | None = None,
                  stream=None, kernel: int = 0) -> torch.Tensor:
    """y = (K + mu I) v (Eq. (1.1)) on the GPU; X (n, d) float64 row-major;
    kernel: AFN_KERNEL_GAUSSIAN or AFN_KERNEL_MATERN32."""
    X = _dev_f64(X, "X").contiguous()
    n, d = X.shape
    vp, nrhs, ldv = _colmajor(v, "v")
    if v.shape[0] != n:
        raise ValueError("v rows != n")
    if out is None:
        out = torch.empty_like(v) if v.dim() == 1 else empty_colmajor(n, nrhs, v.device)
    yp, _, ldy = _colmajor(out, "out")
    if ldv != ldy:
        raise ValueError("v and out must share a leading dimension")
    if kernel == AFN_KERNEL_GAUSSIAN:
        st = lib().kernel_matvec(X.data_ptr(), n, d, l, mu, vp, yp, nrhs, ldv, precision, _stream(stream))
    else:
        st = lib().kernel_matvec_ex(X.data_ptr(), n, d, l, mu, vp, yp, nrhs, ldv, precision, kernel,
                                    _stream(stream))
    _check(st, "kernel_matvec")
    return out


def kernel_matvec_noalloc(X: torch.Tensor, l: float, mu: float, v: torch.Tensor, out: torch.Tensor,
                          precision: int = AFN_FP64, stream=None, kernel: int = 0) -> torch.Tensor:
    """kernel_matvec into a caller-provided out, with the library's static
    scratch array (no device allocation by the library)."""
    X = _dev_f64(X, "X")
    if not X.is_contiguous():
        raise ValueError("X must be contiguous")
    n, d = X.shape
    vp, nrhs, ldv = _colmajor(v, "v")
    yp, _, ldy = _colmajor(out, "out")
    if v.shape[0] != n or out.shape != v.shape or ldv != ldy:
        raise ValueError("v and out must be (n,) or (n, nrhs) with one leading dimension")
    st = lib().kernel_matvec_noalloc(X.data_ptr(), n, d, l, mu, vp, yp, nrhs, ldv, precision, kernel,
                                     _stream(stream))
    _check(st, "kernel_matvec_noalloc")
    return out


@dataclasses.dataclass
class SetupInfo:
    n: int
    d: int
    k: int
    w: int
    rank_r: int
    rank_k_est: int
    rank_eig_branch: int
    rank_eig_count: int
    nnz_g: int
    ms: dict
    method: int = 0
    nu: float = 0.0
    kmv_kept_f64: float = 1.0
    kmv_kept_f32: float = 1.0
    landmarks: int = 1
    kmv_far_f64: float = 0.0
    ws_bytes: int = 0
    ws_bytes_used: int = 0


class Handle:
    """Owns an afn_handle*; afn_destroy runs on close() or garbage collection."""

    def __init__(self, ptr: ctypes.c_void_p, n: int, d: int, ws: torch.Tensor | None = None):
        self._ptr = ptr
        self.n, self.d = n, d
        self.ws = ws      # the workspace the handle's buffers live in (freed after afn_destroy)

    @property
    def ptr(self):
        if not self._ptr:
            raise RuntimeError("handle is closed")
        return self._ptr

    def close(self):
        if self._ptr:
            lib().afn_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> SetupInfo:
        inf = afn_setup_info()
        _check(lib().afn_get_info(self.ptr, ctypes.byref(inf)), "afn_get_info")
        ms = {k: getattr(inf, "ms_" + k) for k in ("rank", "fps", "chol", "knn", "v", "fsai",
                                                   "total")}
        return SetupInfo(inf.n, inf.d, inf.k, inf.w, inf.rank_r, inf.rank_k_est,
                         inf.rank_eig_branch, inf.rank_eig_count, inf.nnz_g, ms, inf.method, inf.nu,
                         inf.kmv_kept_f64, inf.kmv_kept_f32, inf.landmarks, inf.kmv_far_f64,
                         inf.ws_bytes, inf.ws_bytes_used)

    def landmarks(self):
        import numpy as np
        k = self.info().k
        idx = np.zeros(max(k, 1), dtype=np.int32)
        kk = _I64(0)
        _check(lib().afn_get_landmarks(self.ptr, idx.ctypes.data, idx.shape[0], ctypes.byref(kk)),
               "afn_get_landmarks")
        return idx[: kk.value].copy()

    def fsai(self):
        """(rowptr, cols, vals) of G in CSR over the non-landmark points."""
        import numpy as np
        inf = self.info()
        nr = inf.n - inf.k
        rowptr = np.zeros(nr + 1, dtype=np.int64)
        cap = max(int(inf.nnz_g), 1)
        cols = np.zeros(cap, dtype=np.int32)
        vals = np.zeros(cap)
        nnz = _I64(0)
        _check(lib().afn_get_fsai(self.ptr, rowptr.ctypes.data, cols.ctypes.data,
                                  vals.ctypes.data, cap, ctypes.byref(nnz)), "afn_get_fsai")
        return rowptr, cols[: nnz.value].copy(), vals[: nnz.value].copy()

    def cholesky(self):
        import numpy as np
        k = self.info().k
        L = np.zeros((max(k, 1), max(k, 1)), order="F")
        _check(lib().afn_get_cholesky(self.ptr, L.ctypes.data, max(k, 1)), "afn_get_cholesky")
        return L[:k, :k].copy(order="F")


def _params(k=-1, w=64, k_max=2000, m=0, seed=0, precision=AFN_FP64, method=AFN_METHOD_AFN,
            landmarks=AFN_LANDMARKS_AUTO, kernel=0, nrhs_max=0) -> afn_params:
    return afn_params(k=k, k_max=k_max, w=w, m=m, precision=precision, method=method, seed=seed,
                      landmarks=landmarks, kernel=kernel, nrhs_max=nrhs_max, reserved=0)


def afn_workspace_size(n: int, d: int, **params) -> int:
    """Bytes of device workspace afn_setup needs for these sizes (host-only)."""
    prm = _params(**params)
    out = ctypes.c_size_t(0)
    _check(lib().afn_workspace_size(n, d, ctypes.byref(prm), ctypes.byref(out)), "afn_workspace_size")
    return out.value


def afn_setup(X: torch.Tensor, l: float, mu: float, k: int = -1, w: int = 64, k_max: int = 2000,
              m: int = 0, seed: int = 0, precision: int = AFN_FP64, method: int = AFN_METHOD_AFN,
              landmarks: int = AFN_LANDMARKS_AUTO, kernel: int = 0, nrhs_max: int = 64, stream=None,
              ws: torch.Tensor | None = None) -> Handle:
    """Algorithm 2 (landmarks by FPS, chol(K11 + mu I), FSAI of the Schur complement),
    or the Nystrom preconditioner, or Algorithm 5's choice between them (method).
    The handle's device memory is one torch-owned workspace of afn_workspace_size
    bytes (allocated here unless ws is given); the library allocates none."""
    X = _dev_f64(X, "X").contiguous()
    n, d = X.shape
    prm = _params(k=k, k_max=k_max, w=w, m=m, precision=precision, method=method, seed=seed,
                  landmarks=landmarks, kernel=kernel, nrhs_max=nrhs_max)
    need = ctypes.c_size_t(0)
    _check(lib().afn_workspace_size(n, d, ctypes.byref(prm), ctypes.byref(need)), "afn_workspace_size")
    if ws is None:
        ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=X.device)
    if not (ws.is_cuda and ws.dtype == torch.uint8 and ws.is_contiguous()):
        raise TypeError("ws must be a contiguous uint8 CUDA (HIP) tensor")
    h = ctypes.c_void_p()
    _check(lib().afn_setup(X.data_ptr(), n, d, l, mu, ctypes.byref(prm), ws.data_ptr(), ws.numel(),
                           _stream(stream), ctypes.byref(h)), "afn_setup")
    return Handle(h, n, d, ws)


def afn_footprint_bytes(n: int, d: int, k: int = -1, w: int = 64, k_max: int = 2000, m: int = 0,
                        precision: int = AFN_FP64, method: int = AFN_METHOD_AFN, nrhs_max: int = 64) -> int:
    """Device memory of afn_setup for these sizes (= afn_workspace_size; host-only)."""
    return afn_workspace_size(n, d, k=k, w=w, k_max=k_max, m=m, precision=precision, method=method,
                              nrhs_max=nrhs_max)


def afn_apply(h: Handle, r: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
    """z = M^{-1} r (Algorithm 3)."""
    rp, nrhs, ld = _colmajor(r, "r")
    if out is None:
        out = torch.empty_like(r) if r.dim() == 1 else empty_colmajor(r.shape[0], nrhs, r.device)
    zp, _, ldz = _colmajor(out, "out")
    if ldz != ld:
        raise ValueError("r and out must share a leading dimension")
    _check(lib().afn_apply(h.ptr, rp, zp, nrhs, ld, _stream(stream)), "afn_apply")
    return out


def afn_pcg_solve(h: Handle, b: torch.Tensor, tol: float = 1e-6, maxit: int = 500,
                  out: torch.Tensor | None = None, stream=None, allow_noconv: bool = True):
    """PCG from x0 = 0; returns (x, info dict).  ENOCONV is returned in info, not raised,
    when allow_noconv is set."""
    bp, nrhs, ld = _colmajor(b, "b")
    if out is None:
        out = torch.empty_like(b) if b.dim() == 1 else empty_colmajor(b.shape[0], nrhs, b.device)
    xp, _, ldx = _colmajor(out, "out")
    if ldx != ld:
        raise ValueError("b and out must share a leading dimension")
    inf = afn_solve_info()
    ok = (AFN_OK, AFN_ENOCONV, AFN_ESTAGNATION) if allow_noconv else (AFN_OK,)
    st = _check(lib().afn_pcg_solve(h.ptr, bp, xp, nrhs, ld, tol, maxit, ctypes.byref(inf),
                                    _stream(stream)), "afn_pcg_solve", ok)
    return out, dict(status=st, iterations=inf.iterations, converged=bool(inf.converged),
                     relres=inf.relres, relres_true=inf.relres_true, ms_solve=inf.ms_solve,
                     ms_matvec=inf.ms_matvec, matvec_launches=inf.matvec_launches,
                     outer_iterations=inf.outer_iterations, fp64_iterations=inf.fp64_iterations,
                     grouped_units=inf.grouped_units)


class PcgState:
    """A step-wise solve (afn_pcg_begin); release with end()."""

    def __init__(self, ptr: ctypes.c_void_p, handle: Handle, b: torch.Tensor, x: torch.Tensor):
        self._ptr = ptr
        self.handle, self.b, self.x = handle, b, x    # kept alive until the solve ends

    @property
    def ptr(self):
        if not self._ptr:
            raise RuntimeError("state is ended")
        return self._ptr

    def query(self):
        """(done, info dict); info["status"] is the solve's status once done."""
        done = _I32(0)
        inf = afn_solve_info()
        st = lib().afn_pcg_query(self.ptr, ctypes.byref(done), ctypes.byref(inf))
        if st == AFN_EINVAL:
            raise AFNError(st, "afn_pcg_query")
        return bool(done.value), dict(status=st, iterations=inf.iterations, converged=bool(inf.converged),
                                      relres=inf.relres, relres_true=inf.relres_true, ms_solve=inf.ms_solve,
                                      ms_matvec=inf.ms_matvec, matvec_launches=inf.matvec_launches,
                                      outer_iterations=inf.outer_iterations,
                                      fp64_iterations=inf.fp64_iterations, grouped_units=inf.grouped_units)

    def end(self):
        if self._ptr:
            lib().afn_pcg_end(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.end()
        except Exception:
            pass


def afn_pcg_begin(h: Handle, b: torch.Tensor, tol: float = 1e-6, maxit: int = 500,
                  out: torch.Tensor | None = None, stream=None) -> PcgState:
    """Start a step-wise solve of one right-hand side (queued, not waited for)."""
    bp, nrhs, _ = _colmajor(b, "b")
    if nrhs != 1 or b.shape[0] != h.n:
        raise ValueError("b must be one vector of length n")
    if out is None:
        out = torch.empty_like(b)
    xp, _, _ = _colmajor(out, "out")
    ptr = ctypes.c_void_p()
    _check(lib().afn_pcg_begin(h.ptr, bp, xp, tol, maxit, _stream(stream), ctypes.byref(ptr)),
           "afn_pcg_begin")
    return PcgState(ptr, h, b, out)


def afn_pcg_step_many(states, iters: int = 1, stream=None) -> None:
    """Advance every unfinished state by up to iters products with K + mu I,
    one host wait per round for all of them; stream None: each state on the
    stream it was begun on."""
    arr = (ctypes.c_void_p * len(states))(*[s.ptr for s in states])
    sp = ctypes.c_void_p(None) if stream is None else _stream(stream)
    _check(lib().afn_pcg_step_many(arr, len(states), iters, sp), "afn_pcg_step_many")


def group_config(on: bool) -> None:
    """Grouped launches of like solves' iterations in afn_pcg_step_many on or off."""
    lib().afn_group_config(1 if on else 0)


def tune_config(mode: int = AFN_TUNE_OFF, index: int = 0, cache_path: str | None = None) -> None:
    """Autotuner mode (afn_tune_config): AFN_TUNE_OFF, AFN_TUNE_ON or AFN_TUNE_FORCE(index)."""
    _check(lib().afn_tune_config(mode, index, cache_path.encode() if cache_path else None), "afn_tune_config")


def tune_report() -> str:
    """The autotuner's decisions: one line per shape class (key, choice, ms per candidate)."""
    n = _I64(0)
    _check(lib().afn_tune_report(None, 0, ctypes.byref(n)), "afn_tune_report")
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().afn_tune_report(buf, n.value + 1, ctypes.byref(n)), "afn_tune_report")
    return buf.value.decode()
