"""Sketch-and-solve null space on MI355X: Python binding of ``libnsk.so``.

Argument marshalling only: every computation runs in the HIP library behind the C ABI
declared in ``include/nsk.h`` (same names without the ``nsk_`` prefix).  PyTorch supplies
device memory (tensors and workspaces from its caching allocator) and the current HIP
stream.  There is no CPU fallback: if the library is not built, :func:`load` raises.

Main entry points
-----------------
* :func:`sketch`                  -- ``SA = S A`` (line 2 of Algorithm 1).
* :func:`trailing_rsv`            -- Algorithm 1: trailing k right singular vectors.
* :func:`residual`                -- ``|A V_k|_F`` with FP64 accumulation.
* :func:`trailing_rsv_batched`    -- many instances in one persistent launch.
* :func:`tls_solve`, :class:`TLSSketch` -- sketched total least squares and its gradient.
* draw hooks (:func:`philox`, :func:`draw_signs`, ...) for bit-exact checks.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsk.so")

SRHT, SPARSE_SIGN, GAUSSIAN, SRDCT, HRHT = 0, 1, 2, 3, 4
F64, F32, BF16, F8E4M3 = 0, 1, 2, 3
FLAG_RESIDUAL = 1
KINDS = {"srht": SRHT, "sparse": SPARSE_SIGN, "gauss": GAUSSIAN, "srdct": SRDCT, "hrht": HRHT}
STATUS = {0: "ok", 1: "invalid argument", 2: "workspace too small", 3: "Jacobi did not converge",
          4: "HIP runtime error", 5: "unsupported kind/dtype combination"}

_TORCH_DT = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16,
             torch.float8_e4m3fn: F8E4M3}


class NskError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} ({status})")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("zeta", ctypes.c_int32), ("s", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("acc", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("row_groups", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Operand(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("cols", ctypes.c_int64), ("ld", ctypes.c_int64), ("col_exp", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32), ("off", ctypes.c_double),
                ("residual", ctypes.c_double), ("sigma_max", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("k", ctypes.c_int64), ("s", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("Vk", ctypes.c_void_p), ("sigma_k", ctypes.c_void_p), ("info", ctypes.c_void_p)]


INFO_BYTES = ctypes.sizeof(Info)
_lib = None

_P = ctypes.c_void_p
_SIGS = {
    "nsk_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "nsk_version": (ctypes.c_int, []),
    "nsk_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(Desc)]),
    "nsk_sketch": (ctypes.c_int, [ctypes.POINTER(Operand), ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(Desc),
                                  _P, ctypes.c_int64, _P, ctypes.c_size_t, _P]),
    "nsk_trailing_rsv": (ctypes.c_int, [ctypes.POINTER(Operand), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.POINTER(Desc), _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "nsk_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "nsk_trailing_rsv_noalloc": (ctypes.c_int, [ctypes.POINTER(Operand), ctypes.c_int32, ctypes.c_int64,
                                                ctypes.c_int64, ctypes.POINTER(Desc), _P, _P, _P, _P]),
    "nsk_residual": (ctypes.c_int, [ctypes.POINTER(Operand), ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_int64,
                                    _P, _P, ctypes.c_size_t, _P]),
    "nsk_batched_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.POINTER(Desc)]),
    "nsk_trailing_rsv_batched": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.POINTER(Desc), _P,
                                                ctypes.c_size_t, _P]),
    "nsk_autotune_batched": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.POINTER(Desc), _P,
                                            ctypes.c_size_t, _P, ctypes.c_int32]),
    "nsk_tune_lookup": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "nsk_tune_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "nsk_tune_clear": (ctypes.c_int, []),
    "nsk_tls_state_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]),
    "nsk_tls_solve": (ctypes.c_int, [ctypes.POINTER(Operand), ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(Desc),
                                     _P, _P, ctypes.c_size_t, _P, _P, ctypes.c_size_t, _P]),
    "nsk_tls_backward": (ctypes.c_int, [ctypes.POINTER(Desc), ctypes.c_int64, ctypes.c_int64, _P, _P, _P,
                                        ctypes.c_int64, _P, ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    "nsk_profile_enable": (ctypes.c_int, [ctypes.c_int32]),
    "nsk_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    "nsk_philox": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.POINTER(ctypes.c_uint32)]),
    "nsk_tls_solve_multi": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _P, _P, _P, _P, _P,
                                           _P, ctypes.c_size_t, _P]),
    "nsk_null_space": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _P, _P,
                                      _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "nsk_aaa_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, _P]),
    "nsk_aaa": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, _P, _P, _P, _P, _P, _P,
                               ctypes.c_size_t, _P]),
    "nsk_update_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, _P]),
    "nsk_sketch_rows": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, _P, _P, ctypes.c_int64, _P, _P,
                                       ctypes.c_int64, _P, ctypes.c_size_t, _P]),
    "nsk_draw_signs": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, _P]),
    "nsk_draw_srht_rows": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _P]),
    "nsk_draw_sparse": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _P, _P]),
    "nsk_draw_signs_device": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, _P, _P]),
    "nsk_draw_srht_rows_device": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _P, _P]),
    "nsk_draw_sparse_device": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _P,
                                              _P, _P]),
    "nsk_draw_gaussian_device": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_int32, _P, _P]),
}
EXPORTS = tuple(_SIGS)


def load(path: str = LIB_PATH):
    """Load ``libnsk.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnsk.so not built at {path}: run `python -m paper_2206_00975_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(fn, rc):
    if rc != 0:
        raise NskError(fn, rc)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_desc(kind="srht", s=0, seed=0, zeta=8, acc="f64", max_sweeps=0, row_groups=0, flags=0) -> Desc:
    kind_id = KINDS[kind] if isinstance(kind, str) else int(kind)
    acc_id = {"f64": F64, "f32": F32}[acc] if isinstance(acc, str) else int(acc)
    return Desc(kind_id, int(zeta), int(s), int(seed) & 0xFFFFFFFFFFFFFFFF, acc_id, int(max_sweeps),
                int(row_groups), int(flags))


def _blocks(A):
    """Column blocks of a row-major operand: a tensor or a list of tensors (same rows/dtype)."""
    mats = list(A) if isinstance(A, (list, tuple)) else [A]
    ops = (Operand * len(mats))()
    m = None
    keep = []
    for i, t in enumerate(mats):
        exp = None
        if isinstance(t, tuple):          # (fp8 tensor, int8 column exponents)
            t, exp = t
        if t.dim() == 1:
            t = t.unsqueeze(1)
        if t.stride(1) != 1 and t.shape[1] != 1:
            raise ValueError("operand blocks must be row-major with unit column stride")
        if m is None:
            m = t.shape[0]
        elif t.shape[0] != m:
            raise ValueError("column blocks must have the same number of rows")
        ops[i] = Operand(t.data_ptr(), _TORCH_DT[t.dtype], 0, t.shape[1], t.stride(0),
                         exp.data_ptr() if exp is not None else None)
        keep.append((t, exp))
    return ops, len(mats), m, sum(t.shape[1] for t, _ in keep), keep[0][0].device, keep


def workspace_bytes(m, N, k, desc: Desc) -> int:
    return int(load().nsk_workspace_bytes(m, N, k, ctypes.byref(desc)))


def _ws(nbytes, device):
    if nbytes == 0:
        raise NskError("workspace_bytes", 1)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def sketch(A, kind="srht", s=None, seed=0, zeta=8, acc="f64", row_groups=0, out=None):
    """``SA = S A`` as an s x N FP64 tensor on A's device.  ``out``: an s x N FP64 view with unit
    column stride to write into, e.g. columns of a larger sketch (a column update)."""
    lib = load()
    ops, nb, m, N, dev, keep = _blocks(A)
    d = make_desc(kind, s, seed, zeta, acc, row_groups=row_groups)
    ws = _ws(lib.nsk_workspace_bytes(m, N, 1, ctypes.byref(d)), dev)
    if out is None:
        out = torch.empty((s, N), dtype=torch.float64, device=dev)
    elif out.shape != (s, N) or out.dtype != torch.float64 or out.stride(1) != 1:
        raise ValueError("out must be an s x N float64 view with unit column stride")
    _check("nsk_sketch", lib.nsk_sketch(ops, nb, m, ctypes.byref(d), out.data_ptr(), out.stride(0), ws.data_ptr(),
                                        ws.numel(), _stream(dev)))
    return out


def tls_solve_multi(A, B, kind="srdct", s=None, seed=0, zeta=8, acc="f64", max_sweeps=0):
    """TLS with k right-hand sides (Section 4): ``(X, Vk, sigma_k, info)``, X = -V12 V22^{-1}
    (n x k) from the trailing k right singular vectors of the sketched [A | B]."""
    lib = load()
    ops, nb, m, N, dev, keep = _blocks([A, B])
    k = B.shape[1] if B.dim() == 2 else 1
    d = make_desc(kind, s, seed, zeta, acc, max_sweeps)
    ws = _ws(lib.nsk_workspace_bytes(m, N, k, ctypes.byref(d)), dev)
    X = torch.empty((N - k, k), dtype=torch.float64, device=dev)
    Vk = torch.empty((N, k), dtype=torch.float64, device=dev)
    sk = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    _check("nsk_tls_solve_multi", lib.nsk_tls_solve_multi(ops, nb, m, k, ctypes.byref(d), X.data_ptr(), Vk.data_ptr(),
                                                          sk.data_ptr(), info.data_ptr(), ws.data_ptr(), ws.numel(),
                                                          _stream(dev)))
    return X, Vk, sk, info


def null_space(A, eps, kind="srht", s=None, seed=0, zeta=8, acc="f64", relative=True):
    """Epsilon-tolerance Algorithm 1: ``(V, sigma, count)`` with all N right singular vectors of
    SA (columns, non-increasing ``sigma``); the last ``count`` columns have singular values below
    ``eps`` (times the largest when ``relative``)."""
    lib = load()
    ops, nb, m, N, dev, keep = _blocks(A)
    d = make_desc(kind, s, seed, zeta, acc)
    ws = _ws(lib.nsk_workspace_bytes(m, N, N, ctypes.byref(d)), dev)
    V = torch.empty((N, N), dtype=torch.float64, device=dev)
    sigma = torch.empty(N, dtype=torch.float64, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    _check("nsk_null_space", lib.nsk_null_space(ops, nb, m, float(eps), int(bool(relative)), ctypes.byref(d),
                                                V.data_ptr(), sigma.data_ptr(), count.data_ptr(), None,
                                                ws.data_ptr(), ws.numel(), _stream(dev)))
    return V, sigma, count


def aaa(z, f, n_max, tol, kind="srht", s=None, seed=0, zeta=8, ws=None):
    """AAA with a reused sketch (Section 6): ``(support indices, weights, errors)`` for real
    sample points ``z`` and values ``f`` (FP64 device tensors); ``errors[i]`` is the largest
    |f - r| before step i, the last one that of the returned approximant."""
    import numpy as np
    lib = load()
    z = z.contiguous()
    f = f.contiguous()
    if z.dtype != torch.float64 or f.dtype != torch.float64 or z.shape != f.shape or z.dim() != 1:
        raise ValueError("z and f must be FP64 vectors of one length")
    m = z.shape[0]
    s = s if s is not None else 2 * n_max
    d = make_desc(kind, s, seed, zeta)
    need = lib.nsk_aaa_workspace_bytes(m, n_max, ctypes.byref(d))
    if ws is None or ws.numel() < need:
        ws = _ws(need, z.device)
    sup = np.zeros(n_max, dtype=np.int64)
    hist = np.zeros(n_max + 1, dtype=np.float64)
    nsup = ctypes.c_int32(0)
    w = torch.zeros(n_max, dtype=torch.float64, device=z.device)
    _check("nsk_aaa", lib.nsk_aaa(z.data_ptr(), f.data_ptr(), m, n_max, float(tol), ctypes.byref(d), sup.ctypes.data,
                                  w.data_ptr(), ctypes.byref(nsup), hist.ctypes.data, ws.data_ptr(), ws.numel(),
                                  _stream(z.device)))
    n = nsup.value
    return [int(x) for x in sup[:n]], w[:n], [float(x) for x in hist[:n + 1]]


def sketch_rows(SA, values, rows, ops, m, kind="srht", seed=0, zeta=8):
    """Row updates (+1) and downdates (-1) of the sketch ``SA`` (s x N FP64, from a sketch of an
    m-row matrix) in place: ``SA += sum_t ops[t] S_r(:, rows[t]) values[t, :]`` (Section 5)."""
    import numpy as np
    lib = load()
    blks, nb, r, N, dev, keep = _blocks(values)
    d = make_desc(kind, SA.shape[0], seed, zeta)
    idx = np.ascontiguousarray(rows, dtype=np.int64)
    sg = np.ascontiguousarray(ops, dtype=np.int8)
    if idx.size != r or sg.size != r:
        raise ValueError("one row index and one sign per row of values")
    if SA.dtype != torch.float64 or SA.stride(1) != 1 or SA.shape[1] != N:
        raise ValueError("SA must be an s x N float64 tensor with unit column stride")
    ws = _ws(lib.nsk_update_workspace_bytes(r, ctypes.byref(d)), dev)
    _check("nsk_sketch_rows", lib.nsk_sketch_rows(blks, nb, r, idx.ctypes.data, sg.ctypes.data, m, ctypes.byref(d),
                                                  SA.data_ptr(), SA.stride(0), ws.data_ptr(), ws.numel(),
                                                  _stream(dev)))
    return SA


@dataclass
class SolveInfo:
    sweeps: int
    converged: bool
    off: float
    residual: float
    sigma_max: float


def read_info(t: torch.Tensor) -> SolveInfo:
    raw = bytes(t.cpu().numpy().tobytes())
    i = Info.from_buffer_copy(raw)
    return SolveInfo(i.sweeps, bool(i.converged), i.off, i.residual, i.sigma_max)


def trailing_rsv(A, k=1, kind="srht", s=None, seed=0, zeta=8, acc="f64", max_sweeps=0, residual=False,
                 row_groups=0, ws=None, out=None):
    """Algorithm 1.  Returns ``(Vk, sigma_k, info_tensor)``: Vk is N x k FP64, sigma_k k FP64,
    info a raw device buffer (decode with :func:`read_info` after synchronising)."""
    lib = load()
    ops, nb, m, N, dev, keep = _blocks(A)
    d = make_desc(kind, s, seed, zeta, acc, max_sweeps, row_groups, FLAG_RESIDUAL if residual else 0)
    need = lib.nsk_workspace_bytes(m, N, k, ctypes.byref(d))
    if ws is None or ws.numel() < need:
        ws = _ws(need, dev)
    if out is None:
        Vk = torch.empty((N, k), dtype=torch.float64, device=dev)
        sig = torch.empty(k, dtype=torch.float64, device=dev)
        info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    else:
        Vk, sig, info = out
    _check("nsk_trailing_rsv", lib.nsk_trailing_rsv(ops, nb, m, k, ctypes.byref(d), Vk.data_ptr(), sig.data_ptr(),
                                                    info.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev)))
    return Vk, sig, info


def trailing_rsv_noalloc(A, k=1, kind="srht", s=None, seed=0, zeta=8, acc="f64", max_sweeps=0, residual=False,
                         row_groups=0, out=None):
    """:func:`trailing_rsv` on the library's own fixed device array instead of a workspace
    (``nsk_trailing_rsv_noalloc``); ``out = (Vk, sigma_k, info)`` lets the caller supply every
    output so that nothing is allocated."""
    lib = load()
    ops, nb, m, N, dev, keep = _blocks(A)
    d = make_desc(kind, s, seed, zeta, acc, max_sweeps, row_groups, FLAG_RESIDUAL if residual else 0)
    if out is None:
        Vk = torch.empty((N, k), dtype=torch.float64, device=dev)
        sig = torch.empty(k, dtype=torch.float64, device=dev)
        info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    else:
        Vk, sig, info = out
    _check("nsk_trailing_rsv_noalloc", lib.nsk_trailing_rsv_noalloc(ops, nb, m, k, ctypes.byref(d), Vk.data_ptr(),
                                                                    sig.data_ptr(), info.data_ptr(), _stream(dev)))
    return Vk, sig, info


def residual(A, Vk):
    """``|A Vk|_F`` (FP64 accumulation) as a 0-d FP64 tensor."""
    lib = load()
    ops, nb, m, N, dev, keep = _blocks(A)
    Vk = Vk.to(torch.float64).contiguous()
    out = torch.empty((), dtype=torch.float64, device=dev)
    ws = _ws(1024 * 8, dev)
    _check("nsk_residual", lib.nsk_residual(ops, nb, m, Vk.data_ptr(), Vk.shape[1], out.data_ptr(), ws.data_ptr(),
                                            ws.numel(), _stream(dev)))
    return out


def _problems(As, ks, ss, seeds):
    """Problem records and per-instance outputs, carved from three allocations (one each for
    the vectors, the singular values and the info records) rather than three per instance."""
    n = len(As)
    probs = (Problem * n)()
    outs = []
    dev = As[0].device
    shapes = [tuple(A.shape) for A in As]
    vk_all = torch.empty(sum(N * k for (_, N), k in zip(shapes, ks)), dtype=torch.float64, device=dev)
    sig_all = torch.empty(sum(ks), dtype=torch.float64, device=dev)
    info_all = torch.zeros((n, INFO_BYTES), dtype=torch.uint8, device=dev)
    ov = os_ = 0
    for i, A in enumerate(As):
        if A.stride(1) != 1:
            raise ValueError("instances must be row-major")
        m, N = shapes[i]
        Vk = vk_all[ov:ov + N * ks[i]].view(N, ks[i])
        sig = sig_all[os_:os_ + ks[i]]
        info = info_all[i]
        ov += N * ks[i]
        os_ += ks[i]
        probs[i] = Problem(A.data_ptr(), _TORCH_DT[A.dtype], 0, m, N, A.stride(0), ks[i], ss[i],
                           int(seeds[i]) & 0xFFFFFFFFFFFFFFFF, Vk.data_ptr(), sig.data_ptr(), info.data_ptr())
        outs.append((Vk, sig, info))
    return probs, outs


def trailing_rsv_batched(As, ks, ss, seeds, kind="srht", acc="f64", max_sweeps=0, autotune=False, ws=None):
    """Batched Algorithm 1 over a list of row-major instances.  Returns a list of
    ``(Vk, sigma_k, info_tensor)`` per instance."""
    lib = load()
    dev = As[0].device
    probs, outs = _problems(As, ks, ss, seeds)
    d = make_desc(kind, 0, 0, 8, acc, max_sweeps)
    need = lib.nsk_batched_workspace_bytes(probs, len(As), ctypes.byref(d))
    if ws is None or ws.numel() < need:
        ws = _ws(need, dev)
    if autotune:
        big = int(need * 4)
        ws = _ws(big, dev)
        _check("nsk_autotune_batched", lib.nsk_autotune_batched(probs, len(As), ctypes.byref(d), ws.data_ptr(),
                                                                ws.numel(), _stream(dev), 8))
        need = lib.nsk_batched_workspace_bytes(probs, len(As), ctypes.byref(d))
        if ws.numel() < need:
            ws = _ws(need, dev)
    _check("nsk_trailing_rsv_batched", lib.nsk_trailing_rsv_batched(probs, len(As), ctypes.byref(d), ws.data_ptr(),
                                                                    ws.numel(), _stream(dev)))
    return outs


def batched_workspace_bytes(shapes, ks, ss, kind="srht", acc="f64", dtype=torch.float32):
    """Workspace bytes of a batch given shapes (no device memory needed)."""
    lib = load()
    n = len(shapes)
    probs = (Problem * n)()
    for i, (m, N) in enumerate(shapes):
        probs[i] = Problem(1, _TORCH_DT[dtype], 0, m, N, N, ks[i], ss[i], 0, 1, 1, None)
    d = make_desc(kind, 0, 0, 8, acc)
    return int(lib.nsk_batched_workspace_bytes(probs, n, ctypes.byref(d)))


def tune_lookup(n, dtype=torch.float32, acc="f64"):
    return int(load().nsk_tune_lookup(n, _TORCH_DT[dtype], {"f64": F64, "f32": F32}[acc]))


def tune_set(n, rows_per_tile, dtype=torch.float32, acc="f64"):
    _check("nsk_tune_set", load().nsk_tune_set(n, _TORCH_DT[dtype], {"f64": F64, "f32": F32}[acc], rows_per_tile))


def tune_clear():
    load().nsk_tune_clear()


# ------------------------------------------------------------------------------- TLS
def tls_solve(A, b=None, kind="sparse", s=None, seed=0, zeta=8, acc="f64", max_sweeps=0, residual=False,
              ws=None, state=None):
    """Sketched TLS: returns ``(x, state, info)``; ``state`` feeds :func:`tls_backward`."""
    lib = load()
    blocks = [A] if b is None else [A, b.reshape(-1, 1) if b.dim() == 1 else b]
    ops, nb, m, N, dev, keep = _blocks(blocks)
    n = N - 1
    d = make_desc(kind, s, seed, zeta, acc, max_sweeps, flags=FLAG_RESIDUAL if residual else 0)
    need = lib.nsk_workspace_bytes(m, N, 1, ctypes.byref(d))
    if ws is None or ws.numel() < need:
        ws = _ws(need, dev)
    if state is None:
        state = _ws(lib.nsk_tls_state_bytes(n, s, max_sweeps), dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    _check("nsk_tls_solve", lib.nsk_tls_solve(ops, nb, m, ctypes.byref(d), x.data_ptr(), state.data_ptr(),
                                              state.numel(), info.data_ptr(), ws.data_ptr(), ws.numel(),
                                              _stream(dev)))
    return x, state, info


def tls_backward(state, m, n, gx, kind="sparse", s=None, seed=0, zeta=8, acc="f64", out_dtype=torch.float32):
    """Gradient of ``L(x)`` w.r.t. ``[A | b]``: returns ``(dA, db)`` (m x n and m)."""
    lib = load()
    dev = state.device
    d = make_desc(kind, s, seed, zeta, acc)
    ws = _ws(lib.nsk_workspace_bytes(m, n + 1, 1, ctypes.byref(d)), dev)
    gx = gx.to(torch.float64).contiguous()
    dA = torch.empty((m, n), dtype=out_dtype, device=dev)
    db = torch.empty(m, dtype=out_dtype, device=dev)
    _check("nsk_tls_backward", lib.nsk_tls_backward(ctypes.byref(d), m, n, state.data_ptr(), gx.data_ptr(),
                                                    dA.data_ptr(), n, db.data_ptr(), _TORCH_DT[out_dtype],
                                                    ws.data_ptr(), ws.numel(), _stream(dev)))
    return dA, db


class TLSSketch(torch.autograd.Function):
    """``x = TLSSketch.apply(A, b, s, seed, kind, zeta)``: sketched TLS solution (FP64) whose
    backward applies S^T regenerated from the seed and the SVD adjoint of the trailing vector."""

    @staticmethod
    def forward(ctx, A, b, s, seed, kind="sparse", zeta=8):
        x, state, _ = tls_solve(A, b, kind=kind, s=s, seed=seed, zeta=zeta)
        ctx.save_for_backward(state)
        ctx.meta = (A.shape[0], A.shape[1], kind, s, seed, zeta, A.dtype, b.dtype)
        return x

    @staticmethod
    def backward(ctx, gx):
        (state,) = ctx.saved_tensors
        m, n, kind, s, seed, zeta, adt, bdt = ctx.meta
        dA, db = tls_backward(state, m, n, gx, kind=kind, s=s, seed=seed, zeta=zeta, out_dtype=adt)
        return dA, db.to(bdt), None, None, None, None


# ------------------------------------------------------------------------ profiler
PROF_STAGES = ("draws", "sketch", "reduce", "qr", "jacobi", "finish", "post")


def profile_enable(max_calls):
    _check("nsk_profile_enable", load().nsk_profile_enable(max_calls))


def profile_read():
    """Summed milliseconds per stage over the profiled calls and the call count."""
    ms = (ctypes.c_double * len(PROF_STAGES))()
    calls = ctypes.c_int32()
    _check("nsk_profile_read", load().nsk_profile_read(ms, ctypes.byref(calls)))
    return dict(zip(PROF_STAGES, list(ms))), calls.value


# ----------------------------------------------------------------------- draw hooks
def philox(seed, idx, sub, stream):
    out = (ctypes.c_uint32 * 4)()
    _check("nsk_philox", load().nsk_philox(seed, idx, sub, stream, out))
    return list(out)


def draw_signs(seed, m):
    import numpy as np
    d = np.empty(m, dtype=np.int8)
    _check("nsk_draw_signs", load().nsk_draw_signs(seed, m, d.ctypes.data))
    return d


def draw_srht_rows(seed, m, s):
    import numpy as np
    r = np.empty(s, dtype=np.int64)
    _check("nsk_draw_srht_rows", load().nsk_draw_srht_rows(seed, m, s, r.ctypes.data))
    return r


def draw_sparse(seed, m, s, zeta):
    import numpy as np
    rows = np.empty((m, zeta), dtype=np.int32)
    sg = np.empty((m, zeta), dtype=np.int8)
    _check("nsk_draw_sparse", load().nsk_draw_sparse(seed, m, s, zeta, rows.ctypes.data, sg.ctypes.data))
    return rows, sg


def draw_signs_device(seed, m, device="cuda"):
    d = torch.empty(m, dtype=torch.int8, device=device)
    _check("nsk_draw_signs_device", load().nsk_draw_signs_device(seed, m, d.data_ptr(), _stream(d.device)))
    return d


def draw_srht_rows_device(seed, m, s, device="cuda"):
    rows = torch.empty(s, dtype=torch.int32, device=device)
    _check("nsk_draw_srht_rows_device", load().nsk_draw_srht_rows_device(seed, m, s, rows.data_ptr(),
                                                                          _stream(rows.device)))
    return rows


def draw_sparse_device(seed, m, s, zeta, device="cuda"):
    rows = torch.empty((m, zeta), dtype=torch.int32, device=device)
    sg = torch.empty((m, zeta), dtype=torch.int8, device=device)
    _check("nsk_draw_sparse_device", load().nsk_draw_sparse_device(seed, m, s, zeta, rows.data_ptr(), sg.data_ptr(),
                                                                    _stream(rows.device)))
    return rows, sg


def draw_gaussian_device(seed, s, j0, j1, dtype="bf16", device="cuda"):
    dt = {"bf16": BF16, "e4m3": F8E4M3, "f32": F32}[dtype]
    G = torch.empty((s, j1 - j0), dtype=torch.float32, device=device)
    _check("nsk_draw_gaussian_device", load().nsk_draw_gaussian_device(seed, s, j0, j1, dt, G.data_ptr(),
                                                                        _stream(G.device)))
    return G
