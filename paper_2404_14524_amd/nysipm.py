"""Python binding of libnysipm (include/nysipm.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: torch supplies device memory and the current HIP
stream, the library's kernels compute.  There is no CPU fallback: if the
library is not built, or no GPU is visible, the calls raise.
"""

from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnysipm.so")

NYS_OK, NYS_MAXIT = 0, 1
NYS_EINVAL, NYS_ENOMEM, NYS_EHIP, NYS_ENOTPD, NYS_EBREAKDOWN, NYS_ENUMERIC = -1, -2, -3, -4, -5, -6
NYS_F64, NYS_F32, NYS_BF16 = 0, 1, 2
_DT = {torch.float64: NYS_F64, torch.float32: NYS_F32, torch.bfloat16: NYS_BF16}
_SK = {"f64": NYS_F64, "bf16": NYS_BF16, NYS_F64: NYS_F64, NYS_BF16: NYS_BF16}


class NysError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nysipm error {code}: {msg}")
        self.code = code


class nys_matrix(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("ld", C.c_int64), ("dtype", C.c_int),
                ("data", C.c_void_p), ("data_t", C.c_void_p), ("ld_t", C.c_int64),
                ("n_unit", C.c_int64), ("unit_row", C.c_void_p), ("unit_val", C.c_void_p),
                ("tiles", C.c_void_p), ("tiles_t", C.c_void_p)]


class nys_precond(C.Structure):
    _fields_ = [("m", C.c_int64), ("ell", C.c_int32), ("U", C.c_void_p), ("lambda_", C.c_void_p)]


class nys_pchol(C.Structure):
    _fields_ = [("m", C.c_int64), ("ell", C.c_int32), ("piv", C.c_void_p), ("pos", C.c_void_p),
                ("L", C.c_void_p), ("Cinv", C.c_void_p), ("diagS", C.c_void_p)]


class nys_pcg_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("maxit", C.c_int32),
                ("replace_every", C.c_int32), ("poll_every", C.c_int32)]


class nys_pcg_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("true_res", C.c_double),
                ("rel_res", C.c_double)]


class nys_qp(C.Structure):
    _fields_ = [("A", C.POINTER(nys_matrix)), ("A_lo", C.POINTER(nys_matrix)), ("b", C.c_void_p),
                ("c", C.c_void_p), ("q", C.c_void_p), ("vtype", C.c_void_p), ("u", C.c_void_p)]


class nys_ipm_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("ell", C.c_int32),
                ("seed", C.c_uint64), ("sketch_dtype", C.c_int), ("c_nu", C.c_double),
                ("pcg", nys_pcg_opts), ("verbose", C.c_int32), ("no_transposed_copy", C.c_int32),
                ("precond", C.c_int32), ("ell_rule", C.c_int32), ("ell_min", C.c_int32),
                ("ell_max", C.c_int32), ("c_ell", C.c_double), ("reuse_max_age", C.c_int32),
                ("reuse_growth", C.c_double), ("trace", C.c_void_p), ("trace_len", C.c_int32),
                ("separate_corrector", C.c_int32), ("predictor_rtol", C.c_double), ("inner_factor", C.c_double)]


class nys_ipm_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("pcg_iters_total", C.c_int32), ("status", C.c_int32),
                ("kkt_rel", C.c_double), ("rp_rel", C.c_double), ("rd_rel", C.c_double),
                ("mu", C.c_double), ("rho", C.c_double), ("delta", C.c_double),
                ("t_sketch_ms", C.c_double), ("t_pcg_ms", C.c_double), ("t_other_ms", C.c_double),
                ("ru_rel", C.c_double), ("deff_last", C.c_double), ("builds", C.c_int32),
                ("ell_last", C.c_int32)]


EXPORTS = ["nys_create", "nys_destroy", "nys_set_stream", "nys_last_error", "nys_last_timing",
           "nys_profile_enable", "nys_profile_read", "nys_stream_read",
           "nys_normal_apply", "nys_transpose", "nys_test_matrix", "nys_sketch_product", "nys_sketch", "nys_precond_apply",
           "nys_pcg_solve", "nys_newton_solve", "ipm_solve", "ipm_adjoint",
           "nys_pchol_build", "nys_pchol_apply", "nys_pcg_solve_pchol", "ipm_solve_box",
           "nys_deff_estimate", "nys_sketch_size_rule", "nys_precond_rebuild_due", "nys_pcg_solve_noalloc",
           "nys_sketch_tiles_bytes", "nys_sketch_tiles"]

_lib = None
_lock = threading.Lock()
_handles: dict = {}
_streams: dict = {}        # device index -> stream last given to that handle


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libnysipm.so (no GPU needed) and declare the signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_2404_14524_amd.build` "
                              "or __graft_entry__.build(); there is no CPU fallback")
        lib = C.CDLL(path)
        vp, i64, i32, u64, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_double
        pm = C.POINTER(nys_matrix)
        sig = {
            "nys_create": [C.POINTER(vp), C.c_int, vp],
            "nys_destroy": [vp],
            "nys_set_stream": [vp, vp],
            "nys_last_timing": [vp, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl)],
            "nys_profile_enable": [vp, C.c_int],
            "nys_profile_read": [vp, C.c_int, C.POINTER(i64), C.POINTER(dbl)],
            "nys_stream_read": [vp, vp, i64, C.POINTER(dbl)],
            "nys_normal_apply": [vp, pm, vp, dbl, vp, vp],
            "nys_transpose": [vp, pm, vp, i64],
            "nys_test_matrix": [vp, i64, i32, u64, u64, vp],
            "nys_sketch_product": [vp, pm, vp, vp, i32, C.c_int, vp],
            "nys_sketch": [vp, pm, vp, i32, u64, u64, C.c_int, vp, C.POINTER(nys_precond), C.POINTER(dbl)],
            "nys_precond_apply": [vp, C.POINTER(nys_precond), dbl, vp, vp],
            "nys_pcg_solve": [vp, pm, vp, dbl, C.POINTER(nys_precond), vp, vp, C.POINTER(nys_pcg_opts),
                              C.POINTER(nys_pcg_info)],
            "nys_sketch_tiles_bytes": [i64, i64, C.c_int, C.POINTER(i64)],
            "nys_sketch_tiles": [vp, pm, C.c_int, vp],
            "nys_pcg_solve_noalloc": [vp, pm, vp, dbl, C.POINTER(nys_precond), vp, vp,
                                      C.POINTER(nys_pcg_opts), C.POINTER(nys_pcg_info)],
            "nys_pchol_build": [vp, pm, vp, dbl, C.POINTER(nys_pchol)],
            "nys_pchol_apply": [vp, C.POINTER(nys_pchol), vp, vp],
            "nys_pcg_solve_pchol": [vp, pm, vp, dbl, C.POINTER(nys_pchol), vp, vp, C.POINTER(nys_pcg_opts),
                                    C.POINTER(nys_pcg_info)],
            "nys_newton_solve": [vp, pm, vp, vp, vp, dbl, dbl, C.POINTER(nys_precond), vp, vp, vp,
                                 C.POINTER(nys_pcg_opts), vp, vp, vp, C.POINTER(nys_pcg_info)],
            "ipm_solve": [vp, C.POINTER(nys_qp), C.POINTER(nys_ipm_opts), vp, vp, vp,
                          C.POINTER(nys_ipm_info)],
            "ipm_solve_box": [vp, C.POINTER(nys_qp), C.POINTER(nys_ipm_opts), vp, vp, vp, vp, vp,
                              C.POINTER(nys_ipm_info)],
            "ipm_adjoint": [vp, C.POINTER(nys_qp), C.POINTER(nys_ipm_opts), vp, vp, vp, dbl, dbl, vp,
                            vp, vp, vp, vp, C.POINTER(nys_pcg_info)],
            "nys_deff_estimate": [vp, vp, i32, dbl, C.POINTER(dbl)],
            "nys_sketch_size_rule": [i32, dbl, dbl, dbl, i32, i32, i32, i32, dbl],
            "nys_precond_rebuild_due": [i32, i32, i32, i32, i32, dbl],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = C.c_int
        lib.nys_last_error.argtypes = [vp]
        lib.nys_last_error.restype = C.c_char_p
        _lib = lib
        return lib


def _handle(device: torch.device):
    lib = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("nysipm needs a HIP GPU; none is visible (no CPU fallback)")
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _handles.get(idx)
    if h is None:
        h = C.c_void_p()
        rc = lib.nys_create(C.byref(h), idx, None)
        if rc != 0:
            raise NysError(rc, f"nys_create failed on device {idx}")
        _handles[idx] = h
    stream = torch.cuda.current_stream(idx).cuda_stream
    if _streams.get(idx) != stream:
        # nys_set_stream waits for the handle's previous stream (its workspace
        # may still be in use there), so it is called only when torch's
        # current stream changes: calls that only enqueue stay asynchronous
        lib.nys_set_stream(h, C.c_void_p(stream))
        _streams[idx] = stream
    return lib, h


def _check(lib, h, rc: int, allow=(NYS_OK, NYS_MAXIT)):
    if rc not in allow:
        raise NysError(rc, lib.nys_last_error(h).decode())
    return rc


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _vec(t: torch.Tensor, n: int, name: str, device) -> torch.Tensor:
    if t.dtype != torch.float64 or t.device != device or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous float64 tensor of {n} elements on {device}")
    return t


def _mat64(t: torch.Tensor, rows: int, cols: int, name: str, device) -> torch.Tensor:
    """A contiguous float64 rows x cols tensor on `device` (the library reads
    and writes such arguments as dense row-major blocks)."""
    if (t.dtype != torch.float64 or t.device != device or t.dim() != 2 or tuple(t.shape) != (rows, cols)
            or not t.is_contiguous()):
        raise ValueError(f"{name}: need a contiguous float64 tensor of shape ({rows}, {cols}) on {device}")
    return t


def _idx32(t: torch.Tensor, n: int, name: str, device) -> torch.Tensor:
    if t.dtype != torch.int32 or t.device != device or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous int32 tensor of {n} elements on {device}")
    return t


def _units(A: torch.Tensor, units) -> tuple:
    """(count, rows pointer, values pointer) of the unit columns: units is None
    or (rows int32, vals float64), device tensors of equal length (rows
    strictly increasing within [0, m), checked by the library)."""
    if units is None:
        return 0, None, None
    rows, vals = units
    if (rows.dtype != torch.int32 or vals.dtype != torch.float64 or rows.dim() != 1 or vals.dim() != 1
            or rows.numel() != vals.numel() or rows.device != A.device or vals.device != A.device
            or not rows.is_contiguous() or not vals.is_contiguous()):
        raise ValueError("units: need (int32 rows, float64 values), 1-D contiguous, equal length, on A's device")
    k = rows.numel()
    return k, (rows.data_ptr() if k else None), (vals.data_ptr() if k else None)


def ncols(A: torch.Tensor, units=None) -> int:
    """Number of variables: dense columns plus unit columns."""
    return A.shape[1] + (0 if units is None else units[0].numel())


def _rows_ok(T) -> bool:
    """Row-major with a leading dimension the library can take: unit stride
    along a row, and rows that do not overlap (an expanded or broadcast view,
    with row stride 0, would make the kernels read past its storage)."""
    r, c = T.shape
    return (T.stride(1) == 1 or c <= 1) and (T.stride(0) >= c or r <= 1)


def _mat(A: torch.Tensor, A_t: Optional[torch.Tensor] = None, units=None, tiles=None) -> nys_matrix:
    """nys_matrix view of a row-major CUDA tensor; A_t (optional) is the same
    matrix transposed, n x m row-major (see nys_transpose); units (optional)
    appends unit columns (see _units); tiles (optional) is the pair of sketch
    tiles (of A, of A^T) from nys_sketch_tiles."""
    if (A.dim() != 2 or A.dtype not in _DT or not A.is_cuda or not _rows_ok(A)):
        raise ValueError("A: need a 2-D row-major float64/float32/bfloat16 CUDA tensor "
                         "(unit column stride, row stride >= columns)")
    tp, tld = None, 0
    if A_t is not None:
        if (A_t.dim() != 2 or tuple(A_t.shape) != (A.shape[1], A.shape[0]) or A_t.dtype != A.dtype
                or A_t.device != A.device or not _rows_ok(A_t)):
            raise ValueError("A_t: need an n x m row-major tensor of A's dtype on A's device")
        tp, tld = A_t.data_ptr(), max(A_t.stride(0), A.shape[0], 1)
    k, ur, uv = _units(A, units)
    t0 = t1 = None
    if tiles is not None:
        T, Tt = tiles
        for X, tr in ((T, 0), (Tt, 1)):
            if (not isinstance(X, torch.Tensor) or X.dtype != torch.uint8 or X.device != A.device
                    or not X.is_contiguous() or X.numel() != nys_sketch_tiles_bytes(A.shape[0], A.shape[1], tr)):
                raise ValueError("tiles: need the pair (of A, of A^T) made by nys_sketch_tiles for this A")
        t0, t1 = T.data_ptr(), Tt.data_ptr()
    return nys_matrix(A.shape[0], A.shape[1], max(A.stride(0), A.shape[1], 1), _DT[A.dtype],
                      A.data_ptr(), tp, tld, k, ur, uv, t0, t1)


def nys_sketch_tiles_bytes(m: int, n: int, transposed: int) -> int:
    lib = load_library()
    b = C.c_int64(0)
    rc = lib.nys_sketch_tiles_bytes(int(m), int(n), int(transposed), C.byref(b))
    if rc != NYS_OK:
        raise NysError(rc, "nys_sketch_tiles_bytes: bad arguments")
    return b.value


def nys_sketch_tiles(A: torch.Tensor, transposed: bool = False) -> torch.Tensor:
    """Sketch tiles of A (transposed=False) or of A^T (True) as a uint8 device
    tensor; the BF16 sketch reads the pair (tiles of A, tiles of A^T)."""
    lib, h = _handle(A.device)
    nb = nys_sketch_tiles_bytes(A.shape[0], A.shape[1], int(transposed))
    out = torch.empty(max(nb, 16), dtype=torch.uint8, device=A.device)[:nb]
    Am = _mat(A)
    _check(lib, h, lib.nys_sketch_tiles(h, C.byref(Am), int(transposed), C.c_void_p(out.data_ptr())))
    return out


@dataclass
class Precond:
    U: torch.Tensor        # m x ell float64, orthonormal columns
    lam: torch.Tensor      # ell float64, descending
    nu: float = 0.0

    def c(self) -> nys_precond:
        if self.U.dim() != 2:
            raise ValueError("U: need an m x ell tensor")
        m, ell = self.U.shape
        _mat64(self.U, m, ell, "U", self.U.device)
        _vec(self.lam, ell, "lam", self.U.device)
        return nys_precond(m, ell, self.U.data_ptr(), self.lam.data_ptr())


@dataclass
class PChol:
    """Partial Cholesky preconditioner (the Chol-IP-PMM comparator); see nys_pchol."""
    piv: torch.Tensor      # ell int32, ascending pivot rows
    pos: torch.Tensor      # m int32, position in piv or -1
    L: torch.Tensor        # m x ell float64: [L11; L21] in the original row order
    Cinv: torch.Tensor     # ell x ell float64, upper: L11^{-T}
    diagS: torch.Tensor    # m float64

    def c(self) -> nys_pchol:
        if self.L.dim() != 2:
            raise ValueError("L: need an m x ell tensor")
        m, ell = self.L.shape
        dev = self.L.device
        _mat64(self.L, m, ell, "L", dev)
        _mat64(self.Cinv, ell, ell, "Cinv", dev)
        _vec(self.diagS, m, "diagS", dev)
        _idx32(self.piv, ell, "piv", dev)
        _idx32(self.pos, m, "pos", dev)
        return nys_pchol(m, ell, self.piv.data_ptr(), self.pos.data_ptr(),
                         self.L.data_ptr(), self.Cinv.data_ptr(), self.diagS.data_ptr())


def nys_pchol_build(A: torch.Tensor, d: torch.Tensor, delta: float, ell: int, units=None) -> PChol:
    lib, h = _handle(A.device)
    m = A.shape[0]
    _vec(d, ncols(A, units), "d", A.device)
    dev = A.device
    P = PChol(torch.empty(ell, dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.int32, device=dev),
              torch.empty((m, ell), dtype=torch.float64, device=dev),
              torch.empty((ell, ell), dtype=torch.float64, device=dev), torch.empty(m, dtype=torch.float64, device=dev))
    Pc = P.c()
    Am = _mat(A, units=units)
    _check(lib, h, lib.nys_pchol_build(h, C.byref(Am), _ptr(d), float(delta), C.byref(Pc)))
    return P


def nys_pchol_apply(P: PChol, r: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    lib, h = _handle(r.device)
    m = P.L.shape[0]
    _vec(r, m, "r", r.device)
    out = torch.empty_like(r) if out is None else _vec(out, m, "out", r.device)
    Pc = P.c()
    _check(lib, h, lib.nys_pchol_apply(h, C.byref(Pc), _ptr(r), _ptr(out)))
    return out


def _pcg_opts(rtol=1e-10, atol=0.0, maxit=0, replace_every=0, poll_every=0) -> nys_pcg_opts:
    return nys_pcg_opts(rtol, atol, maxit, replace_every, poll_every)


def nys_transpose(A: torch.Tensor) -> torch.Tensor:
    """A^T as a new n x m row-major tensor (the layout nys_matrix.data_t takes),
    written by the library's transpose kernel."""
    lib, h = _handle(A.device)
    m, n = A.shape
    per = 128 // A.element_size()          # 128-byte row pitch
    ld = max((m + per - 1) // per * per, 1)
    buf = torch.empty((n, ld), dtype=A.dtype, device=A.device)
    Am = _mat(A)
    _check(lib, h, lib.nys_transpose(h, C.byref(Am), _ptr(buf), ld))
    return buf[:, :m]


def nys_normal_apply(A: torch.Tensor, d: torch.Tensor, delta: float, v: torch.Tensor,
                     out: Optional[torch.Tensor] = None, A_t: Optional[torch.Tensor] = None,
                     units=None) -> torch.Tensor:
    lib, h = _handle(A.device)
    m = A.shape[0]
    _vec(d, ncols(A, units), "d", A.device)
    _vec(v, m, "v", A.device)
    out = torch.empty(m, dtype=torch.float64, device=A.device) if out is None else _vec(out, m, "out", A.device)
    Am = _mat(A, A_t, units)
    _check(lib, h, lib.nys_normal_apply(h, C.byref(Am), _ptr(d), float(delta), _ptr(v), _ptr(out)))
    return out


def nys_test_matrix(m: int, ell: int, seed: int, counter: int, device="cuda") -> torch.Tensor:
    device = torch.device(device)
    lib, h = _handle(device)
    out = torch.empty((m, ell), dtype=torch.float64, device=device)
    _check(lib, h, lib.nys_test_matrix(h, m, ell, seed, counter, _ptr(out)))
    return out


def nys_sketch_product(A: torch.Tensor, d: torch.Tensor, omega: torch.Tensor, sketch_dtype="f64",
                       out: Optional[torch.Tensor] = None, A_t: Optional[torch.Tensor] = None,
                       units=None, tiles=None) -> torch.Tensor:
    lib, h = _handle(A.device)
    m = A.shape[0]
    if omega.dim() != 2:
        raise ValueError("omega: need an m x ell tensor")
    ell = omega.shape[1]
    _vec(d, ncols(A, units), "d", A.device)
    _mat64(omega, m, ell, "omega", A.device)
    Y = torch.empty((m, ell), dtype=torch.float64, device=A.device) if out is None else out
    _mat64(Y, m, ell, "out", A.device)
    Am = _mat(A, A_t, units, tiles)
    _check(lib, h, lib.nys_sketch_product(h, C.byref(Am), _ptr(d), _ptr(omega), ell, _SK[sketch_dtype],
                                          _ptr(Y)))
    return Y


def nys_sketch(A: torch.Tensor, d: torch.Tensor, ell: int, seed: int = 0, counter: int = 0,
               sketch_dtype="f64", omega: Optional[torch.Tensor] = None,
               A_t: Optional[torch.Tensor] = None, units=None, tiles=None) -> Precond:
    lib, h = _handle(A.device)
    m = A.shape[0]
    _vec(d, ncols(A, units), "d", A.device)
    if omega is not None:
        _mat64(omega, m, ell, "omega", A.device)
    U = torch.empty((m, ell), dtype=torch.float64, device=A.device)
    lam = torch.empty(ell, dtype=torch.float64, device=A.device)
    P = nys_precond(m, ell, U.data_ptr(), lam.data_ptr())
    nu = C.c_double(0.0)
    Am = _mat(A, A_t, units, tiles)
    _check(lib, h, lib.nys_sketch(h, C.byref(Am), _ptr(d), ell, seed, counter, _SK[sketch_dtype],
                                  _ptr(omega), C.byref(P), C.byref(nu)))
    return Precond(U, lam, nu.value)


def nys_precond_apply(P: Precond, delta: float, r: torch.Tensor,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
    lib, h = _handle(r.device)
    m = P.U.shape[0]
    _vec(r, m, "r", r.device)
    out = torch.empty_like(r) if out is None else _vec(out, m, "out", r.device)
    Pc = P.c()
    _check(lib, h, lib.nys_precond_apply(h, C.byref(Pc), float(delta), _ptr(r), _ptr(out)))
    return out


def nys_pcg_solve(A: torch.Tensor, d: torch.Tensor, delta: float, rhs: torch.Tensor,
                  P: Optional[Precond] = None, y0: Optional[torch.Tensor] = None,
                  A_t: Optional[torch.Tensor] = None, units=None, **opts):
    lib, h = _handle(A.device)
    m = A.shape[0]
    _vec(d, ncols(A, units), "d", A.device)
    _vec(rhs, m, "rhs", A.device)
    y = torch.zeros(m, dtype=torch.float64, device=A.device) if y0 is None else _vec(y0, m, "y0", A.device).clone()
    Am = _mat(A, A_t, units)
    o = _pcg_opts(**opts)
    info = nys_pcg_info()
    Pc = P.c() if P is not None else None
    if isinstance(P, PChol):
        rc = lib.nys_pcg_solve_pchol(h, C.byref(Am), _ptr(d), float(delta), C.byref(Pc), _ptr(rhs), _ptr(y),
                                     C.byref(o), C.byref(info))
    else:
        rc = lib.nys_pcg_solve(h, C.byref(Am), _ptr(d), float(delta), C.byref(Pc) if Pc else None,
                               _ptr(rhs), _ptr(y), C.byref(o), C.byref(info))
    _check(lib, h, rc)
    return y, info


def nys_pcg_solve_noalloc(A: torch.Tensor, d: torch.Tensor, delta: float, rhs: torch.Tensor,
                          y: torch.Tensor, P: Optional[Precond] = None, A_t: Optional[torch.Tensor] = None,
                          units=None, **opts):
    """nys_pcg_solve without any device allocation: y (m FP64, caller-owned)
    holds the initial guess and receives the solution in place; the library
    works in its fixed per-GPU scratch array.  The binding allocates nothing
    on the device either."""
    lib, h = _handle(A.device)
    m = A.shape[0]
    _vec(d, ncols(A, units), "d", A.device)
    _vec(rhs, m, "rhs", A.device)
    _vec(y, m, "y", A.device)
    Am = _mat(A, A_t, units)
    o = _pcg_opts(**opts)
    info = nys_pcg_info()
    Pc = P.c() if P is not None else None
    rc = lib.nys_pcg_solve_noalloc(h, C.byref(Am), _ptr(d), float(delta), C.byref(Pc) if Pc else None,
                                   _ptr(rhs), _ptr(y), C.byref(o), C.byref(info))
    _check(lib, h, rc)
    return y, info


def nys_newton_solve(A, q, x, z, rho, delta, r_d, r_p, r_xz, P: Optional[Precond] = None,
                     A_t: Optional[torch.Tensor] = None, units=None, **opts):
    lib, h = _handle(A.device)
    m, n = A.shape[0], ncols(A, units)
    dev = A.device
    for t, k, nm in ((q, n, "q"), (x, n, "x"), (z, n, "z"), (r_d, n, "r_d"), (r_p, m, "r_p"),
                     (r_xz, n, "r_xz")):
        _vec(t, k, nm, dev)
    dx = torch.empty(n, dtype=torch.float64, device=dev)
    dz = torch.empty(n, dtype=torch.float64, device=dev)
    dy = torch.empty(m, dtype=torch.float64, device=dev)
    Am = _mat(A, A_t, units)
    o = _pcg_opts(**opts)
    info = nys_pcg_info()
    Pc = P.c() if P is not None else None
    rc = lib.nys_newton_solve(h, C.byref(Am), _ptr(q), _ptr(x), _ptr(z), float(rho), float(delta),
                              C.byref(Pc) if Pc else None, _ptr(r_d), _ptr(r_p), _ptr(r_xz), C.byref(o),
                              _ptr(dx), _ptr(dy), _ptr(dz), C.byref(info))
    _check(lib, h, rc)
    return dx, dy, dz, info


PRECONDS = {"nystrom": 0, "none": 1, "pchol": 2}
ELL_RULES = {"fixed": 0, "deff": 1, "theorem": 2}
# fields of one record of the per-iteration trace (NYS_TR_*)
TRACE_FIELDS = ("k", "mu", "delta", "ell", "built", "d_hat", "lam_last", "pcg", "rule_d_hat", "rule_lam_last",
                "rp_rel", "rd_rel", "time_ms")


def _ipm_opts(ell, tol=1e-6, max_iter=100, seed=0, sketch_dtype="f64", c_nu=1.0, verbose=False,
              pcg_rtol=0.0, pcg_maxit=0, replace_every=0, poll_every=0,
              transposed_copy=True, precond="nystrom", ell_rule="fixed", ell_min=0, ell_max=0,
              c_ell=0.0, reuse_max_age=0, reuse_growth=0.0, trace=None, separate_corrector=False,
              predictor_rtol=0.0, inner_factor=0.0) -> nys_ipm_opts:
    """trace: None, or a C-contiguous float64 numpy array of shape
    (L, len(TRACE_FIELDS)) that receives one record per IP-PMM iteration k < L."""
    tp, tl = None, 0
    if trace is not None:
        if (not isinstance(trace, np.ndarray) or trace.dtype != np.float64 or trace.ndim != 2
                or trace.shape[1] != len(TRACE_FIELDS) or not trace.flags.c_contiguous):
            raise ValueError(f"trace: need a C-contiguous float64 numpy array of shape (L, {len(TRACE_FIELDS)})")
        tp, tl = trace.ctypes.data, trace.shape[0]
    return nys_ipm_opts(tol, max_iter, ell, seed, _SK[sketch_dtype], c_nu,
                        _pcg_opts(pcg_rtol, 0.0, pcg_maxit, replace_every, poll_every), int(verbose),
                        0 if transposed_copy else 1, PRECONDS[precond], ELL_RULES[ell_rule], ell_min,
                        ell_max, c_ell, reuse_max_age, reuse_growth, tp, tl, int(bool(separate_corrector)),
                        predictor_rtol, inner_factor)


def nys_deff_estimate(lam: torch.Tensor, mu: float) -> float:
    """sum_i lam_i / (lam_i + mu) over the Nystrom eigenvalues lam (device)."""
    lib, h = _handle(lam.device)
    _vec(lam, lam.numel(), "lam", lam.device)
    out = C.c_double()
    _check(lib, h, lib.nys_deff_estimate(h, _ptr(lam), lam.numel(), float(mu), C.byref(out)))
    return out.value


def nys_sketch_size_rule(rule: str, d_hat: float, lam_last: float, mu: float, k: int, ell_prev: int,
                         ell_min: int, ell_max: int, c_ell: float = 2.0) -> int:
    """Sketch size for the preconditioner built at IP-PMM iteration k (host)."""
    lib = load_library()
    r = lib.nys_sketch_size_rule(ELL_RULES[rule], float(d_hat), float(lam_last), float(mu), int(k),
                                 int(ell_prev), int(ell_min), int(ell_max), float(c_ell))
    if r < 0:
        raise NysError(r, "nys_sketch_size_rule: bad rule or clamps")
    return r


def nys_precond_rebuild_due(k: int, k_build: int, pcg_prev: int, pcg_ref: int, max_age: int,
                            growth: float) -> bool:
    """The reuse rule: True when the preconditioner is built anew at iteration k (host)."""
    lib = load_library()
    return bool(lib.nys_precond_rebuild_due(int(k), int(k_build), int(pcg_prev), int(pcg_ref), int(max_age),
                                            float(growth)))


def _qp(A, b, c, q, A_lo, A_t=None, vtype=None, u=None, units=None):
    Am = _mat(A, A_t, units)
    Alo = _mat(A_lo) if A_lo is not None else None
    keep = (Am, Alo)
    qp = nys_qp(C.pointer(Am), C.pointer(Alo) if Alo is not None else None, b.data_ptr(),
                c.data_ptr(), q.data_ptr(), _ptr(vtype), _ptr(u))
    return qp, keep


VAR_NONNEG, VAR_FREE, VAR_BOX = 0, 1, 2


def ipm_solve_box(A: torch.Tensor, b: torch.Tensor, c: torch.Tensor, q: torch.Tensor, vtype: torch.Tensor,
                  u: torch.Tensor, ell: int, A_lo: Optional[torch.Tensor] = None,
                  A_t: Optional[torch.Tensor] = None, units=None, **kw):
    """Nys-IP-PMM for free (VAR_FREE), non-negative (VAR_NONNEG) and box-constrained
    (VAR_BOX, 0 <= x_j <= u_j) variables.  vtype: n int8; u: n float64 (read on
    box indices).  units: optional unit columns (see _units) after the dense
    ones.  Returns (x, y, z, w, s, info)."""
    lib, h = _handle(A.device)
    m, n = A.shape[0], ncols(A, units)
    dev = A.device
    _vec(b, m, "b", dev)
    _vec(c, n, "c", dev)
    _vec(q, n, "q", dev)
    _vec(u, n, "u", dev)
    if vtype.dtype != torch.int8 or vtype.numel() != n or not vtype.is_contiguous() or vtype.device != dev:
        raise ValueError(f"vtype: need a contiguous int8 tensor of {n} elements on {dev}")
    x, z, w, s = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4))
    y = torch.empty(m, dtype=torch.float64, device=dev)
    qp, keep = _qp(A, b, c, q, A_lo, A_t, vtype, u, units)
    o = _ipm_opts(ell, **kw)
    info = nys_ipm_info()
    rc = lib.ipm_solve_box(h, C.byref(qp), C.byref(o), _ptr(x), _ptr(y), _ptr(z), _ptr(w), _ptr(s), C.byref(info))
    _check(lib, h, rc)
    del keep
    return x, y, z, w, s, info


def ipm_solve(A: torch.Tensor, b: torch.Tensor, c: torch.Tensor, q: torch.Tensor, ell: int,
              A_lo: Optional[torch.Tensor] = None, A_t: Optional[torch.Tensor] = None, units=None, **kw):
    """Nys-IP-PMM.  Returns (x, y, z, info: nys_ipm_info).  Without A_t the
    library makes its own transposed copy of A unless transposed_copy=False.
    units: optional unit columns (see _units) after the dense ones."""
    lib, h = _handle(A.device)
    m, n = A.shape[0], ncols(A, units)
    dev = A.device
    _vec(b, m, "b", dev)
    _vec(c, n, "c", dev)
    _vec(q, n, "q", dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    z = torch.empty(n, dtype=torch.float64, device=dev)
    y = torch.empty(m, dtype=torch.float64, device=dev)
    qp, keep = _qp(A, b, c, q, A_lo, A_t, units=units)
    o = _ipm_opts(ell, **kw)
    info = nys_ipm_info()
    rc = lib.ipm_solve(h, C.byref(qp), C.byref(o), _ptr(x), _ptr(y), _ptr(z), C.byref(info))
    _check(lib, h, rc)
    del keep
    return x, y, z, info


def ipm_adjoint(A, b, c, q, x, y, z, rho, delta, g, ell, A_lo=None, want=("c", "b", "q", "A"),
                A_t=None, units=None, **kw):
    """Gradients of L with dL/dx = g through the KKT conditions.  Returns
    (dict of requested gradients, nys_pcg_info).  (The library rejects unit
    columns here.)"""
    lib, h = _handle(A.device)
    m, n = A.shape[0], ncols(A, units)
    dev = A.device
    for t, k, nm in ((b, m, "b"), (c, n, "c"), (q, n, "q"), (x, n, "x"), (z, n, "z"), (y, m, "y"),
                     (g, n, "g")):
        _vec(t, k, nm, dev)
    out = {}
    if "c" in want:
        out["c"] = torch.empty(n, dtype=torch.float64, device=dev)
    if "b" in want:
        out["b"] = torch.empty(m, dtype=torch.float64, device=dev)
    if "q" in want:
        out["q"] = torch.empty(n, dtype=torch.float64, device=dev)
    if "A" in want:
        out["A"] = torch.empty((m, n), dtype=torch.float64, device=dev)
    qp, keep = _qp(A, b, c, q, A_lo, A_t, units=units)
    kw.pop("tol", None)
    o = _ipm_opts(ell, **kw)
    info = nys_pcg_info()
    rc = lib.ipm_adjoint(h, C.byref(qp), C.byref(o), _ptr(x), _ptr(y), _ptr(z), float(rho), float(delta),
                         _ptr(g), _ptr(out.get("c")), _ptr(out.get("b")), _ptr(out.get("q")),
                         _ptr(out.get("A")), C.byref(info))
    _check(lib, h, rc)
    del keep
    return out, info


def nys_last_timing(device="cuda"):
    lib, h = _handle(torch.device(device))
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib.nys_last_timing(h, C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


KERNEL_CLASSES = {"normal_pass1": 0, "normal_pass2": 1, "sketch_w": 2, "sketch_y": 3, "gemm_f64": 4}


def nys_profile_enable(enable: bool = True, device="cuda"):
    """Start (and reset) or stop HIP-event timing of the library's kernel classes."""
    lib, h = _handle(torch.device(device))
    _check(lib, h, lib.nys_profile_enable(h, int(bool(enable))))


def nys_profile_read(device="cuda") -> dict:
    """{class name: (launches, total milliseconds)} since nys_profile_enable."""
    lib, h = _handle(torch.device(device))
    out = {}
    for name, k in KERNEL_CLASSES.items():
        n, ms = C.c_int64(), C.c_double()
        _check(lib, h, lib.nys_profile_read(h, k, C.byref(n), C.byref(ms)))
        out[name] = (int(n.value), float(ms.value))
    return out


def nys_stream_read(t: torch.Tensor) -> float:
    """Milliseconds for one 16-byte non-temporal read of the tensor's bytes
    (read-stream reference for roofline reports)."""
    lib, h = _handle(t.device)
    if not t.is_contiguous():
        raise ValueError("nys_stream_read: need a contiguous tensor")
    nbytes = t.numel() * t.element_size()
    ms = C.c_double()
    _check(lib, h, lib.nys_stream_read(h, C.c_void_p(t.data_ptr()), nbytes - nbytes % 16, C.byref(ms)))
    return ms.value
