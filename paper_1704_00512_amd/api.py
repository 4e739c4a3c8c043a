"""Python face of the C interface (include/chess.h), one function per entry
point, same names.  PyTorch supplies device memory and the stream; every
computation happens in libchess.so.

Matrices are passed as (pattern, values): a BlockPattern holds device int64
row_ptr / int32 col_idx tensors, values are float64 device tensors of shape
[nnzb, b, b] (each block row-major).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

_OPT_FIELDS = {name for name, _ in _lib.chess_opts._fields_}


class ChessError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_lib.ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = _lib.ERRORS.get(code, str(code))


@dataclass
class BlockPattern:
    """A block sparsity pattern resident on the GPU."""
    b: int
    nb: int
    row_ptr: torch.Tensor  # int64 [nb+1], device
    col_idx: torch.Tensor  # int32 [nnzb], device

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    @staticmethod
    def from_host(b: int, row_ptr, col_idx, device="cuda") -> "BlockPattern":
        rp = torch.as_tensor(np.asarray(row_ptr, dtype=np.int64), device=device)
        ci = torch.as_tensor(np.asarray(col_idx, dtype=np.int32), device=device)
        return BlockPattern(b=int(b), nb=int(rp.shape[0] - 1), row_ptr=rp, col_idx=ci)

    def c(self) -> _lib.chess_pattern:
        rp, ci = self.row_ptr, self.col_idx
        if rp.dtype != torch.int64 or ci.dtype != torch.int32:
            raise ValueError("pattern row_ptr must be int64 and col_idx int32")
        if not (rp.is_cuda and ci.is_cuda and rp.is_contiguous() and ci.is_contiguous()):
            raise ValueError("pattern row_ptr / col_idx must be contiguous CUDA tensors")
        if rp.dim() != 1 or ci.dim() != 1 or rp.shape[0] != self.nb + 1:
            raise ValueError(f"pattern row_ptr shape {tuple(rp.shape)} != ({self.nb + 1},)")
        return _lib.chess_pattern(self.b, self.nb, self.nnzb, self.row_ptr.data_ptr(),
                                  self.col_idx.data_ptr())

    def zeros(self) -> torch.Tensor:
        return torch.zeros((self.nnzb, self.b, self.b), dtype=torch.float64,
                           device=self.row_ptr.device)


def _mat(p: BlockPattern, val: torch.Tensor) -> _lib.chess_matrix:
    if val.dtype != torch.float64 or not val.is_cuda or not val.is_contiguous():
        raise ValueError("matrix values must be a contiguous float64 CUDA tensor")
    if tuple(val.shape) != (p.nnzb, p.b, p.b):
        raise ValueError(f"values shape {tuple(val.shape)} != {(p.nnzb, p.b, p.b)}")
    return _lib.chess_matrix(p.c(), val.data_ptr(), _lib.CHESS_F64)


def _check_x(pattern: BlockPattern, opts: dict):
    # a warm-start S^-1/2 lives on the kernel pattern
    for k in ("sinvhalf_in", "sinvhalf_out"):
        v = opts.get(k)
        if v is not None and tuple(v.shape) != (pattern.nnzb, pattern.b, pattern.b):
            raise ValueError(f"{k} shape {tuple(v.shape)} != {(pattern.nnzb, pattern.b, pattern.b)}")


def default_opts(**kw) -> _lib.chess_opts:
    o = _lib.chess_opts()
    _lib.load().chess_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k not in _OPT_FIELDS:
            raise TypeError(f"unknown option {k}")
        if k in ("bounds", "s_bounds", "mu_bracket"):
            arr = getattr(o, k)
            arr[0], arr[1] = (math.nan, math.nan) if v is None else (float(v[0]), float(v[1]))
        elif k == "mu":
            o.mu = math.nan if v is None else float(v)
        elif k == "precision" and isinstance(v, str):
            o.precision = {"f64": _lib.CHESS_F64, "f32": _lib.CHESS_F32, "bf16": _lib.CHESS_BF16,
                           "bf16x3": _lib.CHESS_BF16X3}[v]
        elif k == "smearing" and isinstance(v, str):
            o.smearing = {"erfc": _lib.CHESS_ERFC, "fermi_dirac": _lib.CHESS_FERMI_DIRAC}[v]
        elif k in ("sinvhalf_in", "sinvhalf_out"):
            # a float64 CUDA tensor on the kernel pattern, kept alive by the caller
            if v is not None and (v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous()):
                raise ValueError(f"{k} must be a contiguous float64 CUDA tensor")
            setattr(o, k, None if v is None else v.data_ptr())
        elif k == "bounds_mode" and isinstance(v, str):
            o.bounds_mode = {"gershgorin": 0, "lanczos": 1, "learned": 2, "learned_lanczos": 3}[v]
        else:
            setattr(o, k, v)
    return o


class Context:
    """A chess_ctx on one device, ordered on torch's current stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self._L = _lib.load()
        torch.cuda.set_device(device)
        st = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = st
        h = ctypes.c_void_p()
        rc = self._L.chess_create(ctypes.byref(h), device, ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise ChessError(rc, "chess_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.chess_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != 0:
            raise ChessError(rc, self._L.chess_last_error(self._h).decode())

    def set_progress(self, fn, every: int = 256):
        """Calls fn(stage: str, done: int, total: int) every `every` chain
        products (after a stream wait); fn=None switches it off."""
        if fn is None:
            self._progress = None
            self._check(self._L.chess_set_progress(self._h, _lib.PROGRESS_FN(), None, 0))
            return

        def trampoline(_user, stage, done, total):
            fn(stage.decode(), int(done), int(total))

        self._progress = _lib.PROGRESS_FN(trampoline)  # kept alive with the context
        self._check(self._L.chess_set_progress(self._h, self._progress, None, int(every)))


def chess_fermi_operator(ctx: Context, H: torch.Tensor, pat_h: BlockPattern, S: torch.Tensor,
                         pat_s: BlockPattern, pattern: BlockPattern, n_electrons: float,
                         kT: float, out: torch.Tensor | None = None, **opts):
    K = pattern.zeros() if out is None else out
    info = _lib.chess_info()
    _check_x(pattern, opts)
    o = default_opts(**opts)
    mh, ms, mk, pk = _mat(pat_h, H), _mat(pat_s, S), _mat(pattern, K), pattern.c()
    ctx._check(ctx._L.chess_fermi_operator(ctx._h, ctypes.byref(mh), ctypes.byref(ms),
                                           ctypes.byref(pk), float(n_electrons), float(kT),
                                           ctypes.byref(mk), ctypes.byref(info), ctypes.byref(o)))
    return K, info.as_dict()


def chess_matrix_power(ctx: Context, S: torch.Tensor, pat_s: BlockPattern, a: float,
                       pattern: BlockPattern, out: torch.Tensor | None = None, **opts):
    R = pattern.zeros() if out is None else out
    info = _lib.chess_info()
    o = default_opts(**opts)
    ms, mr, pk = _mat(pat_s, S), _mat(pattern, R), pattern.c()
    ctx._check(ctx._L.chess_matrix_power(ctx._h, ctypes.byref(ms), float(a), ctypes.byref(pk),
                                         ctypes.byref(mr), ctypes.byref(info), ctypes.byref(o)))
    return R, info.as_dict()


def chess_eigs_in_interval(ctx: Context, H: torch.Tensor, pat_h: BlockPattern, S: torch.Tensor,
                           pat_s: BlockPattern, lo: float, hi: float, pattern: BlockPattern,
                           capacity: int = 1 << 16, **opts):
    buf = (ctypes.c_double * max(capacity, 1))()
    nf = ctypes.c_int64(0)
    info = _lib.chess_info()
    _check_x(pattern, opts)
    o = default_opts(**opts)
    mh, ms, pk = _mat(pat_h, H), _mat(pat_s, S), pattern.c()
    rc = ctx._L.chess_eigs_in_interval(ctx._h, ctypes.byref(mh), ctypes.byref(ms), float(lo),
                                       float(hi), ctypes.byref(pk), buf, int(capacity),
                                       ctypes.byref(nf), ctypes.byref(info), ctypes.byref(o))
    ctx._check(rc)
    return np.array(buf[: nf.value], dtype=np.float64), info.as_dict()


def chess_chebyshev(ctx: Context, M: torch.Tensor, pat_m: BlockPattern, lo: float, hi: float,
                    pattern: BlockPattern, n_pl: int, coef=None, want_moments: bool = True,
                    **opts):
    coef = np.zeros((0, n_pl)) if coef is None else np.atleast_2d(np.asarray(coef, dtype=np.float64))
    nq = coef.shape[0]
    if nq and coef.shape[1] != n_pl:
        raise ValueError("coefficient sets must have n_pl entries")
    accs = [pattern.zeros() for _ in range(nq)]
    arr = (_lib.chess_matrix * max(nq, 1))()
    for q in range(nq):
        arr[q] = _mat(pattern, accs[q])
    cbuf = np.ascontiguousarray(coef.ravel()) if nq else np.zeros(1)
    mom = np.zeros(n_pl)
    o = default_opts(**opts)
    mm, pk = _mat(pat_m, M), pattern.c()
    ctx._check(ctx._L.chess_chebyshev(
        ctx._h, ctypes.byref(mm), float(lo), float(hi), ctypes.byref(pk), int(n_pl), int(nq),
        cbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), arr if nq else None,
        mom.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_moments else None,
        ctypes.byref(o)))
    return accs, mom


def chess_masked_product(ctx: Context, A: torch.Tensor, pat_a: BlockPattern, B: torch.Tensor,
                         pat_b: BlockPattern, pat_c: BlockPattern, out: torch.Tensor | None = None):
    C = pat_c.zeros() if out is None else out
    ma, mb, mc = _mat(pat_a, A), _mat(pat_b, B), _mat(pat_c, C)
    ctx._check(ctx._L.chess_masked_product(ctx._h, ctypes.byref(ma), ctypes.byref(mb),
                                           ctypes.byref(mc)))
    return C


# ---------------------------------------------------------------------------
# learned predictor of bounds and mu
# ---------------------------------------------------------------------------

def chess_features(ctx: Context, H: torch.Tensor, pat_h: BlockPattern, S: torch.Tensor,
                   pat_s: BlockPattern, pattern: BlockPattern, n_electrons: float, kT: float,
                   **opts):
    """(features [64] float32 numpy, Gershgorin interval of H' (lo, hi))."""
    f = np.zeros(_lib.N_FEATURES, dtype=np.float32)
    g = np.zeros(2)
    mh, ms, pk = _mat(pat_h, H), _mat(pat_s, S), pattern.c()
    o = default_opts(**opts)
    ctx._check(ctx._L.chess_features(
        ctx._h, ctypes.byref(mh), ctypes.byref(ms), ctypes.byref(pk), float(n_electrons),
        float(kT), f.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
        g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(o)))
    return f, (float(g[0]), float(g[1]))


def _fptr(t: torch.Tensor | None):
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def chess_mlp_forward(ctx: Context, params: torch.Tensor, x: torch.Tensor,
                      norm: torch.Tensor | None = None, want_hidden: bool = False):
    """y [B, 3] (and the hidden activations [B, 128] if want_hidden)."""
    B = x.shape[0]
    y = torch.empty((B, _lib.MLP_OUT), dtype=torch.float32, device=x.device)
    hid = torch.empty((B, _lib.MLP_HIDDEN), dtype=torch.float32, device=x.device) if want_hidden else None
    ctx._check(ctx._L.chess_mlp_forward(ctx._h, _fptr(params), _fptr(norm), _fptr(x), int(B),
                                        _fptr(hid), _fptr(y)))
    return (y, hid) if want_hidden else y


def chess_mlp_grad(ctx: Context, params, x, hidden, y, target, work=None, grad=None,
                   want_loss: bool = True):
    """(grad [CHESS_MLP_PARAMS], loss or None)."""
    B = x.shape[0]
    if work is None:
        work = torch.empty(B * (_lib.MLP_OUT + _lib.MLP_HIDDEN), dtype=torch.float32, device=x.device)
    if grad is None:
        grad = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = ctypes.c_double(float("nan"))
    ctx._check(ctx._L.chess_mlp_grad(ctx._h, _fptr(params), _fptr(x), _fptr(hidden), _fptr(y),
                                     _fptr(target), int(B), _fptr(work), _fptr(grad),
                                     ctypes.byref(loss) if want_loss else None))
    return grad, (loss.value if want_loss else None)


def chess_mlp_grad_noalloc(ctx: Context, params, x, hidden, y, target, grad=None,
                           want_loss: bool = True):
    """As chess_mlp_grad with the library's fixed workspace (no device
    allocation inside the call; pass `grad` to allocate nothing here either).
    (grad, loss or None)."""
    B = x.shape[0]
    if grad is None:
        grad = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = ctypes.c_double(float("nan"))
    ctx._check(ctx._L.chess_mlp_grad_noalloc(ctx._h, _fptr(params), _fptr(x), _fptr(hidden), _fptr(y),
                                             _fptr(target), int(B), _fptr(grad),
                                             ctypes.byref(loss) if want_loss else None))
    return grad, (loss.value if want_loss else None)


def chess_mlp_adam(ctx: Context, params, grad, m, v, step: int, lr: float, beta1=0.9,
                   beta2=0.999, eps=1e-8):
    ctx._check(ctx._L.chess_mlp_adam(ctx._h, _fptr(params), _fptr(grad), _fptr(m), _fptr(v),
                                     int(params.numel()), float(lr), float(beta1), float(beta2),
                                     float(eps), int(step)))


def chess_model_load(ctx: Context, blob: np.ndarray):
    b = np.ascontiguousarray(blob, dtype=np.float32)
    ctx._check(ctx._L.chess_model_load(ctx._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                       int(b.size)))


def chess_model_save(ctx: Context) -> np.ndarray:
    b = np.zeros(_lib.MODEL_FLOATS, dtype=np.float32)
    rc = ctx._L.chess_model_save(ctx._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(b.size))
    if rc != 0:
        raise ChessError(rc, "no model loaded")
    return b


# ---------------------------------------------------------------------------
# batches of independent systems
# ---------------------------------------------------------------------------

def chess_fermi_operator_batched(ctx: Context, systems, want_k=(True, True, True),
                                 want_sinvhalf: bool = True, want_sinv: bool = True, **opts):
    """systems: list of dicts with H, pat_h, S, pat_s, pattern, n_electrons,
    kT and optionally mu_trial (3 values; NaN / missing: predicted).
    Returns one dict per system: K (list of 3 tensors or None), Sinvhalf,
    Sinv, ne_trial (3 floats), info."""
    n = len(systems)
    items = (_lib.chess_batch_item * n)()
    keep = []  # ctypes objects that must outlive the call
    outs = []
    for i, sy in enumerate(systems):
        pk = sy["pattern"]
        mh, ms, pc = _mat(sy["pat_h"], sy["H"]), _mat(sy["pat_s"], sy["S"]), pk.c()
        it = items[i]
        it.H, it.S, it.pattern = ctypes.pointer(mh), ctypes.pointer(ms), ctypes.pointer(pc)
        it.n_electrons, it.kT = float(sy["n_electrons"]), float(sy["kT"])
        mt = sy.get("mu_trial", (float("nan"),) * 3)
        for q in range(3):
            it.mu_trial[q] = float(mt[q])
        res = dict(K=[None] * 3, Sinvhalf=None, Sinv=None)
        mats = []
        for q in range(3):
            if want_k[q]:
                res["K"][q] = pk.zeros()
                m = _mat(pk, res["K"][q])
                it.K_out[q] = ctypes.pointer(m)
                mats.append(m)
        if want_sinvhalf:
            res["Sinvhalf"] = pk.zeros()
            m = _mat(pk, res["Sinvhalf"])
            it.Sinvhalf_out = ctypes.pointer(m)
            mats.append(m)
        if want_sinv:
            res["Sinv"] = pk.zeros()
            m = _mat(pk, res["Sinv"])
            it.Sinv_out = ctypes.pointer(m)
            mats.append(m)
        ne = (ctypes.c_double * 3)()
        info = _lib.chess_info()
        it.ne_trial = ctypes.cast(ne, ctypes.POINTER(ctypes.c_double))
        it.info = ctypes.pointer(info)
        keep += [mh, ms, pc, ne, info] + mats
        outs.append((res, ne, info))
    o = default_opts(**opts)
    ctx._check(ctx._L.chess_fermi_operator_batched(ctx._h, n, items, ctypes.byref(o)))
    result = []
    for res, ne, info in outs:
        res["ne_trial"] = [ne[0], ne[1], ne[2]]
        res["info"] = info.as_dict()
        result.append(res)
    return result


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def chess_ssf_to_bcsr(b: int, n: int, keyg, val, keyv=None):
    """Segment Storage Format -> block CSR (host numpy arrays, see chess.h):
    keyg [nseg, 4] (c_s, c_e, r_s, r_e, 1-based), val (1-D), keyv (1-based
    starts or None).  Returns (row_ptr int64, col_idx int32, values [nnzb, b, b])."""
    L = _lib.load()
    keyg = np.ascontiguousarray(np.asarray(keyg, dtype=np.int64).reshape(-1, 4))
    val = np.ascontiguousarray(np.asarray(val, dtype=np.float64).ravel())
    kv = None if keyv is None else np.ascontiguousarray(np.asarray(keyv, dtype=np.int64))
    if kv is not None and kv.size != keyg.shape[0]:
        raise ValueError("keyv needs one entry per segment")
    nnzb = ctypes.c_int64(0)
    args = (int(b), int(n), keyg.shape[0], _ptr(keyg), _ptr(kv), _ptr(val), val.size)
    rc = L.chess_ssf_to_bcsr(*args, None, None, None, 0, ctypes.byref(nnzb))
    if rc != 0:
        raise ChessError(rc, "chess_ssf_to_bcsr: malformed segments")
    rp = np.zeros(n // b + 1, dtype=np.int64)
    ci = np.zeros(max(nnzb.value, 1), dtype=np.int32)
    vb = np.zeros((max(nnzb.value, 1), b, b), dtype=np.float64)
    rc = L.chess_ssf_to_bcsr(*args, _ptr(rp), _ptr(ci), _ptr(vb), nnzb.value, ctypes.byref(nnzb))
    if rc != 0:
        raise ChessError(rc, "chess_ssf_to_bcsr failed")
    return rp, ci[:nnzb.value], vb[:nnzb.value]


def chess_bcsr_to_ssf(b: int, row_ptr, col_idx, val):
    """Block CSR -> Segment Storage Format (host numpy arrays, see chess.h).
    Returns (keyg [nseg, 4], keyv [nseg], values)."""
    L = _lib.load()
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    ci = np.ascontiguousarray(np.asarray(col_idx, dtype=np.int32))
    vb = np.ascontiguousarray(np.asarray(val, dtype=np.float64))
    nb = rp.size - 1
    if vb.size != ci.size * b * b:
        raise ValueError("values must be [nnzb, b, b]")
    nseg, nval = ctypes.c_int64(0), ctypes.c_int64(0)
    head = (int(b), nb, _ptr(rp), _ptr(ci), _ptr(vb))
    rc = L.chess_bcsr_to_ssf(*head, None, None, None, 0, ctypes.byref(nseg), ctypes.byref(nval))
    if rc != 0:
        raise ChessError(rc, "chess_bcsr_to_ssf: malformed pattern")
    kg = np.zeros((max(nseg.value, 1), 4), dtype=np.int64)
    kv = np.zeros(max(nseg.value, 1), dtype=np.int64)
    v = np.zeros(max(nval.value, 1), dtype=np.float64)
    rc = L.chess_bcsr_to_ssf(*head, _ptr(kg), _ptr(kv), _ptr(v), nseg.value, ctypes.byref(nseg),
                             ctypes.byref(nval))
    if rc != 0:
        raise ChessError(rc, "chess_bcsr_to_ssf failed")
    return kg[:nseg.value], kv[:nseg.value], v[:nval.value]


_FN = {"erfc": _lib.CHESS_FN_ERFC, "fermi_dirac": _lib.CHESS_FN_FERMI_DIRAC,
       "power": _lib.CHESS_FN_POWER, "penalty": _lib.CHESS_FN_PENALTY}


def chess_degree(fn: str, param: float, lo: float, hi: float, tol_fit: float) -> int:
    """Eq. 7's degree for an occupation of width param (fn "erfc" or
    "fermi_dirac", centred on [lo, hi]) or for x^param (fn "power"); with fn
    "penalty", the terms with which Eq. 6 is trusted on param rows (lo, hi
    and tol_fit unused).  Host only.  Raises ChessError with the library's
    code."""
    L = _lib.load()
    out = ctypes.c_int32(0)
    rc = L.chess_degree(_FN[fn], float(param), float(lo), float(hi), float(tol_fit),
                        ctypes.byref(out))
    if rc != 0:
        raise ChessError(rc, "chess_degree")
    return int(out.value)
